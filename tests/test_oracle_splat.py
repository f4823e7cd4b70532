"""Pins for the oracle's grid placement and voxelisation (CPU only).

Each check compares the oracle with something it does not compute itself:
closed forms of the Gaussian splat, a brute-force lattice scan, exact rational
arithmetic, conservation of mass and the exact voxel permutation that a 90 degree
rotation about the grid centre induces.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def test_pose_center_is_rounded_centroid():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 7, 20, 61):
        x = rng.integers(-40000, 40000, size=(n, 3)).astype(np.int32)
        c = oracle.pose_center(x)
        for d in range(3):
            mean = Fraction(int(x[:, d].astype(np.int64).sum()), n)
            # nearest integer, halves rounded toward +inf
            want = math.floor(mean + Fraction(1, 2))
            assert int(c[d]) == want


def test_pose_center_halves_round_up():
    x = np.array([[0, 0, 0], [1, -1, 3]], dtype=np.int32)   # means 0.5, -0.5, 1.5
    assert list(oracle.pose_center(x)) == [1, 0, 2]


def test_voxel_centers_symmetric_half_angstrom_offsets():
    c = np.array([100, -7, 3], dtype=np.int64)
    G = 4
    idx = np.arange(G)
    P = oracle.voxel_center(c, G, np.stack([idx] * 3, 1))
    # centres at c + (-1.5, -0.5, 0.5, 1.5) A
    assert list(P[:, 0] - c[0]) == [-1536, -512, 512, 1536]


def _one_atom(X, G, center, feat=None):
    feat = np.ones((1, 19), dtype=np.float32) if feat is None else feat
    return oracle.splat_pose(np.array([X], dtype=np.int32), feat, center, G)


def test_splat_atom_on_voxel_centre_closed_form():
    # G odd -> the centre voxel's centre is the grid centre.  Support = 1 + 6 + 12
    # voxels at distances 0, 1, sqrt(2) A; sqrt(3) A lies beyond 1.5 A.
    G = 9
    c = np.array([5000, -3000, 777], dtype=np.int64)
    g = _one_atom(c, G, c)[..., 0]
    Z = 1.0 + 6.0 * math.exp(-2.0) + 12.0 * math.exp(-4.0)
    m = G // 2
    assert np.count_nonzero(g) == 19
    assert g[m, m, m] == pytest.approx(1.0 / Z, rel=1e-15)
    assert g[m + 1, m, m] == pytest.approx(math.exp(-2.0) / Z, rel=1e-15)
    assert g[m, m - 1, m + 1] == pytest.approx(math.exp(-4.0) / Z, rel=1e-15)
    assert g[m + 1, m + 1, m + 1] == 0.0
    assert 1.0 / Z == pytest.approx(0.4921746, abs=1e-7)


def test_splat_atom_on_voxel_corner_closed_form():
    # Even G: the grid centre is a voxel corner; the 8 surrounding voxels lie at
    # sqrt(0.75) A, the next shell at sqrt(2.75) A > 1.5 A.  Each gets 1/8 (up to the
    # rounding of the normaliser's eight-term sum).
    G = 6
    c = np.array([1024, 2048, -512], dtype=np.int64)
    g = _one_atom(c, G, c)[..., 3]
    assert np.count_nonzero(g) == 8
    nz = g[g != 0]
    np.testing.assert_allclose(nz, 0.125, rtol=4e-16, atol=0)
    assert set(map(tuple, np.argwhere(g))) == {(i, j, k) for i in (2, 3) for j in (2, 3) for k in (2, 3)}


def test_splat_support_matches_brute_force_lattice_scan():
    rng = np.random.default_rng(11)
    G = 8
    c = np.array([0, 0, 0], dtype=np.int64)
    for _ in range(40):
        X = rng.integers(-5000, 5000, size=3)
        g = _one_atom(X, G, c)[..., 0]
        # brute force over an oversized lattice: which voxels are within 1536 u
        sup, inside = [], []
        for i in range(-6, G + 6):
            for j in range(-6, G + 6):
                for k in range(-6, G + 6):
                    P = c + 512 * (2 * np.array([i, j, k]) - G + 1)
                    D = int(((X - P) ** 2).sum())
                    if D <= 1536 * 1536:
                        sup.append(math.exp(-D / 524288.0))
                        if 0 <= i < G and 0 <= j < G and 0 <= k < G:
                            inside.append(((i, j, k), math.exp(-D / 524288.0)))
        Z = math.fsum(sup)
        want = np.zeros((G, G, G))
        for (i, j, k), wv in inside:
            want[i, j, k] = wv / Z
        np.testing.assert_allclose(g, want, rtol=1e-13, atol=1e-16)


def test_splat_mass_conservation():
    b = synth.make_poses("c1", 1, pose0=3)
    G = 24
    c = oracle.pose_center(b.xyz[b.is_lig.astype(bool)])
    g = oracle.splat_pose(b.xyz, b.feat, c, G)
    # atoms whose whole support lies inside the grid keep their unit mass
    inside_mass = np.zeros(19)
    lo = c - 512 * (G - 1)
    hi = c + 512 * (G - 1)
    n_clipped = 0
    for a in range(b.n_atoms):
        X = b.xyz[a].astype(np.int64)
        # support inside iff every candidate voxel within 1536 u is inside the box
        if np.all(X - 1536 >= lo - 512) and np.all(X + 1536 <= hi + 512):
            inside_mass += b.feat[a]
        else:
            n_clipped += 1
    gsum = g.sum(axis=(0, 1, 2))
    # atoms clipped by the grid boundary: bound their mass separately
    full = np.array([oracle.splat_pose(b.xyz[a:a + 1], b.feat[a:a + 1], c, G).sum(axis=(0, 1, 2))
                     for a in range(b.n_atoms)])
    np.testing.assert_allclose(full.sum(0), gsum, rtol=1e-12, atol=1e-12)
    scale = np.abs(b.feat).sum(0) + 1.0
    for a in range(b.n_atoms):
        X = b.xyz[a].astype(np.int64)
        if np.all(X - 1536 >= lo - 512) and np.all(X + 1536 <= hi + 512):
            np.testing.assert_allclose(full[a], b.feat[a], rtol=0, atol=1e-12 * scale.max())
    assert n_clipped < b.n_atoms


def test_splat_mass_conservation_interior_pose():
    # A pose well inside a large grid loses nothing: per-channel grid sums equal the
    # per-channel feature sums.
    b = synth.make_poses("c1", 1, pose0=7)
    c = oracle.pose_center(b.xyz[b.is_lig.astype(bool)])
    g = oracle.splat_pose(b.xyz, b.feat, c, 40)
    want = b.feat.astype(np.float64).sum(0)
    np.testing.assert_allclose(g.sum(axis=(0, 1, 2)), want, rtol=0,
                               atol=1e-12 * np.abs(b.feat).sum())


def _rot90_z(X, c):
    d = X.astype(np.int64) - c
    return np.stack([-d[:, 1], d[:, 0], d[:, 2]], axis=1) + c


def _rot90_x(X, c):
    d = X.astype(np.int64) - c
    return np.stack([d[:, 0], -d[:, 2], d[:, 1]], axis=1) + c


def test_splat_exact_voxel_permutation_under_90deg_rotation():
    b = synth.make_poses("c1", 1, pose0=1)
    G = 24
    c = oracle.pose_center(b.xyz[b.is_lig.astype(bool)])
    g = oracle.splat_pose(b.xyz, b.feat, c, G)
    gz = oracle.splat_pose(_rot90_z(b.xyz, c), b.feat, c, G)
    # (i, j, k) -> (G-1-j, i, k): rotated[G-1-j, i, k] == g[i, j, k], bitwise
    want = np.empty_like(g)
    ii, jj, kk = np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij")
    want[G - 1 - jj, ii, kk] = g[ii, jj, kk]
    assert np.array_equal(gz, want)
    gx = oracle.splat_pose(_rot90_x(b.xyz, c), b.feat, c, G)
    want = np.empty_like(g)
    want[ii, G - 1 - kk, jj] = g[ii, jj, kk]
    assert np.array_equal(gx, want)


def test_splat_atoms_outside_grid_contribute_nothing():
    G = 4
    c = np.zeros(3, dtype=np.int64)
    X = np.array([0, 0, 3 * 1024 + 600])   # > 1.5 A beyond the last voxel centre (1.5 A)
    assert not _one_atom(X, G, c).any()


def test_splat_coincident_high_feature_atoms_closed_form():
    # 100 atoms on one voxel centre with |f| = 64 (signs mixed per channel): the
    # voxel holds the closed-form centre weight 1 / (1 + 6 e^-2 + 12 e^-4) times the
    # feature sum, far beyond what a 2^-20 fixed-point int32 accumulator holds
    # (+-2048), and the mass of every channel is conserved.
    G = 24
    c = np.array([0, 0, 0], np.int64)
    n = 100
    X = np.tile(np.array([[512, 512, 512]], np.int32), (n, 1))      # centre of voxel (12, 12, 12)
    rng = np.random.default_rng(5)
    F = (64.0 * rng.choice([-1.0, 1.0], size=(n, 19))).astype(np.float32)
    F[:, 0] = 64.0                                                   # channel 0: all +64
    g = oracle.splat_pose(X, F, c, G)
    Z = 1.0 + 6.0 * math.exp(-2.0) + 12.0 * math.exp(-4.0)
    np.testing.assert_allclose(g[12, 12, 12], F.astype(np.float64).sum(0) / Z, rtol=1e-13, atol=1e-9)
    assert g[12, 12, 12, 0] > 2048.0
    np.testing.assert_allclose(g.sum(axis=(0, 1, 2)), F.astype(np.float64).sum(0), rtol=0, atol=1e-9)
