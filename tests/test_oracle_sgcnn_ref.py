"""Pins for the oracle's SG-CNN message passing (CPU only).

The SG-CNN is PotentialNet on gated graph sequence networks (Sec. 3.3.1,
Table II): an embedding, K_c rounds over the covalent graph, then K_n rounds
over the non-covalent graph, each round summing neighbour states, applying that
round's message matrix and a GRU shared by the stage, then a gated readout over
ligand atoms.  The references below share nothing with the oracle's code:

* a torch float64 module built from `nn.Linear` and `nn.GRUCell`, whose graphs
  are dense adjacency matrices computed here from the integer coordinates, for
  the tiny, full and paper-shaped models and for a 2 + 2-round model with
  distinct per-round matrices;
* reach: which input atoms can change an atom's final state follows from the
  order of the stages and from which graph each stage uses, so swapping the
  stages' graphs changes the dependence pattern;
* a hand-worked 4-atom pose with 2-wide states whose every intermediate value is
  written out below from the definition (Sec. 3.3.1 via GGNN): neighbour sums as
  explicit index lists, products as explicit dot products.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
import synth

U = 1024   # fixed-point units per Angstrom


class TorchSGCNN(torch.nn.Module):
    """The SG-CNN forward as torch float64 modules over dense adjacency."""

    def __init__(self, arch, w):
        super().__init__()
        t = lambda k: torch.tensor(np.asarray(w[k], np.float64))
        H, Hn, C = arch.H, (arch.H_nc or arch.H), arch.n_ch
        self.arch = arch

        def lin(name, fin, fout, bias=True):
            m = torch.nn.Linear(fin, fout, bias=bias).double()
            m.weight.data = t(name + ".w")
            if bias:
                m.bias.data = t(name + ".b")
            return m

        def gru(stage, width):
            g = torch.nn.GRUCell(width, width).double()
            g.weight_ih.data = t(f"sg.{stage}.gru.w_ih")
            g.weight_hh.data = t(f"sg.{stage}.gru.w_hh")
            g.bias_ih.data = t(f"sg.{stage}.gru.b_ih")
            g.bias_hh.data = t(f"sg.{stage}.gru.b_hh")
            return g

        self.embed = lin("sg.embed", C, H)
        self.msg_c = torch.nn.ModuleList([lin(f"sg.cov.msg{r}", H, H, bias=False) for r in range(arch.K_c)])
        self.gru_c = gru("cov", H)
        if arch.H_nc:
            self.mid_gate = lin("sg.mid.gate", H + C, H)
            self.mid_val = lin("sg.mid.val", H, H)
            self.embed2 = lin("sg.embed2", H, Hn)
        self.msg_n = torch.nn.ModuleList([lin(f"sg.nc.msg{r}", Hn, Hn, bias=False) for r in range(arch.K_n)])
        self.gru_n = gru("nc", Hn)
        self.gate = lin("sg.gate", Hn + (H if arch.H_nc else C), Hn)
        self.val = lin("sg.val", Hn, Hn)

    @staticmethod
    def adjacency(xyz, r_u):
        X = torch.tensor(np.asarray(xyz, np.int64))
        d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
        A = (d2 <= r_u * r_u) & ~torch.eye(X.shape[0], dtype=torch.bool)
        return A.double()

    def forward(self, xyz, feat, is_lig, A_c=None, A_n=None):
        x = torch.tensor(np.asarray(feat, np.float64))
        if A_c is None:
            A_c = self.adjacency(xyz, self.arch.r_cov_u)
        if A_n is None:
            A_n = self.adjacency(xyz, self.arch.r_nc_u)
        h = self.embed(x)
        for msg in self.msg_c:
            h = self.gru_c(msg(A_c @ h), h)
        u = x
        if self.arch.H_nc:
            g = torch.sigmoid(self.mid_gate(torch.cat([h, x], 1))) * self.mid_val(h)
            h, u = self.embed2(g), g
        for msg in self.msg_n:
            h = self.gru_n(msg(A_n @ h), h)
        lig = torch.tensor(np.asarray(is_lig).astype(bool))
        s = (torch.sigmoid(self.gate(torch.cat([h, u], 1))) * self.val(h))[lig].sum(0)
        return s, h


def _oracle(b, w, arch):
    cov = oracle.radius_graph_pose(b.xyz, arch.r_cov_u)
    nc = oracle.radius_graph_pose(b.xyz, arch.r_nc_u)
    return oracle.sgcnn_pose(b.feat, b.is_lig, cov, nc, w, arch, return_h=True)


def _two_two(arch_name):
    """The named model with two covalent and two non-covalent rounds."""
    base = synth.ARCHS[arch_name]
    return dataclasses.replace(base, name=f"{arch_name}_2x2", K_c=2, K_n=2)


@pytest.mark.parametrize("arch_name,cfg,pose", [("tiny", "c1", 3), ("full", "c2", 2), ("paper", "c2", 5),
                                                ("tiny_2x2", "c1", 7), ("paper_2x2", "c1", 1)])
def test_sgcnn_matches_torch_modules_over_dense_adjacency(arch_name, cfg, pose):
    arch = _two_two(arch_name[:-4]) if arch_name.endswith("_2x2") else synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    b = synth.make_poses(cfg, 1, pose0=pose)
    s, h = _oracle(b, w, arch)
    with torch.no_grad():
        ts, th = TorchSGCNN(arch, w)(b.xyz, b.feat, b.is_lig)
    # the graphs must be non-trivial for the comparison to reach the rounds
    A_c = TorchSGCNN.adjacency(b.xyz, arch.r_cov_u)
    A_n = TorchSGCNN.adjacency(b.xyz, arch.r_nc_u)
    assert A_c.sum() > 10 and A_n.sum() > 5 * A_c.sum()
    np.testing.assert_allclose(h, th.numpy(), rtol=1e-11, atol=1e-12 * np.abs(th.numpy()).max())
    np.testing.assert_allclose(s, ts.numpy(), rtol=1e-11, atol=1e-12 * np.abs(ts.numpy()).max())


def test_sgcnn_round_matrices_are_applied_in_round_order():
    # swapping the two covalent message matrices (and, separately, the two
    # non-covalent ones) must change the result: each round has its own matrix
    arch = _two_two("tiny")
    w = synth.make_weights(arch)
    b = synth.make_poses("c1", 1, pose0=7)
    s0, _ = _oracle(b, w, arch)
    for stage in ("cov", "nc"):
        w2 = dict(w)
        w2[f"sg.{stage}.msg0.w"], w2[f"sg.{stage}.msg1.w"] = w[f"sg.{stage}.msg1.w"], w[f"sg.{stage}.msg0.w"]
        s1, _ = _oracle(b, w2, arch)
        with torch.no_grad():
            ts, _ = TorchSGCNN(arch, w2)(b.xyz, b.feat, b.is_lig)
        np.testing.assert_allclose(s1, ts.numpy(), rtol=1e-11, atol=1e-12 * np.abs(s1).max())
        assert np.abs(s1 - s0).max() > 1e-6 * np.abs(s0).max()


def _chain_pose():
    """Four atoms on the x axis at 0, 3.2, 4.7 and 7.9 A: with cutoffs 1.6 / 4.5 A
    the covalent graph is {1-2} and the non-covalent graph {0-1, 1-2, 2-3}."""
    xs = [0.0, 3.2, 4.7, 7.9]
    xyz = np.array([[int(round(x * U)), 0, 0] for x in xs], np.int32)
    return xyz


def test_sgcnn_reach_follows_stage_order_and_graphs():
    # One covalent round then one non-covalent round: atom 0's final state depends
    # on atoms {0, 1, 2} (2 reaches 1 in the covalent round, 1 reaches 0 in the
    # non-covalent round) and not on atom 3.  Running the stages in the other
    # order, or giving each stage the other's graph, gives {0, 1} instead.
    arch = dataclasses.replace(synth.ARCHS["tiny"], name="reach", K_c=1, K_n=1)
    w = synth.make_weights(arch)
    xyz = _chain_pose()
    cov = oracle.radius_graph_pose(xyz, arch.r_cov_u)
    nc = oracle.radius_graph_pose(xyz, arch.r_nc_u)
    assert list(cov[1]) == [2, 1] and list(nc[1]) == [1, 0, 2, 1, 3, 2]
    rng = np.random.default_rng(11)
    feat = rng.standard_normal((4, 19))
    lig = np.ones(4, np.uint8)
    _, h0 = oracle.sgcnn_pose(feat, lig, cov, nc, w, arch, return_h=True)
    depends = []
    for j in range(4):
        f2 = feat.copy()
        f2[j] += rng.standard_normal(19)
        _, h1 = oracle.sgcnn_pose(f2, lig, cov, nc, w, arch, return_h=True)
        depends.append(bool(np.abs(h1[0] - h0[0]).max() > 0))
    assert depends == [True, True, True, False]


def test_sgcnn_hand_worked_four_atom_pose():
    # H = 2, K_c = K_n = 2, the chain pose above (covalent {1-2}, non-covalent
    # {0-1, 1-2, 2-3}).  Each quantity below is computed from the definition with
    # explicit neighbour lists and dot products.
    H, C = 2, 19
    arch = dataclasses.replace(synth.ARCHS["tiny"], name="hand", H=H, K_c=2, K_n=2)
    w = {}
    E = np.zeros((H, C))
    E[0, 0], E[1, 1], E[0, 18], E[1, 18] = 0.5, -0.25, 0.1, 0.2
    w["sg.embed.w"], w["sg.embed.b"] = E, np.array([0.05, -0.05])
    # four distinct, non-symmetric message matrices
    M = {("cov", 0): [[1.0, 0.5], [0.0, 1.0]], ("cov", 1): [[0.0, 1.0], [-1.0, 0.25]],
         ("nc", 0): [[0.5, 0.0], [0.75, -0.5]], ("nc", 1): [[1.0, -1.0], [0.5, 0.5]]}
    for (st, r), m in M.items():
        w[f"sg.{st}.msg{r}.w"] = np.array(m)
    G = {}
    rng = np.random.default_rng(5)
    for st in ("cov", "nc"):
        G[st] = dict(w_ih=np.round(rng.standard_normal((3 * H, H)), 2),
                     w_hh=np.round(rng.standard_normal((3 * H, H)), 2),
                     b_ih=np.round(rng.standard_normal(3 * H) * 0.1, 2),
                     b_hh=np.round(rng.standard_normal(3 * H) * 0.1, 2))
        for k, v in G[st].items():
            w[f"sg.{st}.gru.{k}"] = v
    w["sg.gate.w"] = np.round(rng.standard_normal((H, H + C)) * 0.5, 2)
    w["sg.gate.b"] = np.array([0.1, -0.1])
    w["sg.val.w"] = np.array([[1.0, 2.0], [-1.0, 0.5]])
    w["sg.val.b"] = np.array([0.0, 0.3])
    xyz = _chain_pose()
    feat = np.zeros((4, C))
    feat[:, 0] = [1, 0, 1, 0]
    feat[:, 1] = [0, 1, 0, 1]
    feat[:, 18] = [1, 1, -1, -1]
    lig = np.array([1, 1, 0, 0], np.uint8)

    def dot(a, b):
        return sum(float(x) * float(y) for x, y in zip(a, b))

    def matvec(Mx, v):
        return [dot(row, v) for row in Mx]

    def sig(x):
        return 1.0 / (1.0 + math.exp(-x))

    def gru(g, m, h):
        gi = [dot(g["w_ih"][k], m) + g["b_ih"][k] for k in range(3 * H)]
        gh = [dot(g["w_hh"][k], h) + g["b_hh"][k] for k in range(3 * H)]
        out = []
        for c in range(H):
            r = sig(gi[c] + gh[c])
            z = sig(gi[H + c] + gh[H + c])
            n = math.tanh(gi[2 * H + c] + r * gh[2 * H + c])
            out.append((1 - z) * n + z * h[c])
        return out

    nbr = {"cov": {0: [], 1: [2], 2: [1], 3: []}, "nc": {0: [1], 1: [0, 2], 2: [1, 3], 3: [2]}}
    h = [[dot(E[c], feat[i]) + w["sg.embed.b"][c] for c in range(H)] for i in range(4)]
    for st in ("cov", "nc"):
        for r in range(2):
            a = [[sum(h[j][c] for j in nbr[st][i]) for c in range(H)] for i in range(4)]
            h = [gru(G[st], matvec(M[(st, r)], a[i]), h[i]) for i in range(4)]
    s = [0.0] * H
    for i in (0, 1):
        gate_in = list(h[i]) + list(feat[i])
        for c in range(H):
            s[c] += sig(dot(w["sg.gate.w"][c], gate_in) + w["sg.gate.b"][c]) * \
                (dot(w["sg.val.w"][c], h[i]) + w["sg.val.b"][c])
    cov = oracle.radius_graph_pose(xyz, arch.r_cov_u)
    nc = oracle.radius_graph_pose(xyz, arch.r_nc_u)
    got_s, got_h = oracle.sgcnn_pose(feat, lig, cov, nc, w, arch, return_h=True)
    np.testing.assert_allclose(got_h, np.array(h), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(got_s, np.array(s), rtol=1e-13, atol=1e-14)
