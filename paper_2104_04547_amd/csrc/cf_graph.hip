// Covalent and non-covalent neighbour lists by exact integer distance tests.
//
// The SG-CNN reads a spatial graph with two edge types chosen by distance
// threshold (Sec. 1; thresholds are hyper-parameters, Table I / Table II).  An
// edge (i, j) exists for i != j in the same pose when |x_i - x_j|^2 <= r^2 with
// coordinates and r in 2^-10 A integers, so the lists are exact.
//
// Design: one workgroup per pose, one thread per atom i (rounds of 256), and an
// all-pairs sweep over j in ascending order: the j coordinates come from a small
// LDS tile that every lane reads at the same address (a broadcast), so the sweep
// is a stream of independent integer tests, and the columns of each row come out
// ascending with no sort.  For the pose sizes of docking (hundreds of atoms) the
// n^2 tests cost less than a cell grid would (which tests ~27 cells of candidates
// per atom and needs the whole pose plus the grid in LDS).  Pass 1 counts degrees,
// a single-workgroup scan turns per-pose totals into edge offsets, and pass 2
// repeats the sweep and writes each row in order.
//
// Exactness: a pose whose coordinates span less than 2^31 units on every axis
// (any real complex) takes 32-bit differences and an unsigned 64-bit sum of
// squares (< 3 * 2^62); a wider pose takes 64-bit differences and a box test
// (|d| <= r on each axis, r <= 2^16) before squaring.
#include <climits>

#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 1024;  // atoms of the j tile in LDS (16 KB)

struct GraphShared {
  int4 tile[kTile];
  int red[kThreads / 64][6];
  int scan_tmp[kThreads];
  int wide;
};

__device__ inline int block_excl_scan(int v, int *tmp, int *total) {
  // inclusive scan over kThreads values via LDS (Hillis-Steele), returns exclusive
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const int t = threadIdx.x >= o ? tmp[threadIdx.x - o] : 0;
    __syncthreads();
    tmp[threadIdx.x] += t;
    __syncthreads();
  }
  const int incl = tmp[threadIdx.x];
  *total = tmp[kThreads - 1];
  __syncthreads();
  return incl - v;
}

// 1 when some axis of the pose spans 2^31 units or more (all threads get the answer)
__device__ int pose_is_wide(GraphShared &S, const int32_t *__restrict__ xyz, int a0, int n) {
  int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
  for (int i = threadIdx.x; i < n; i += kThreads)
    for (int d = 0; d < 3; ++d) {
      const int x = xyz[3 * (int64_t)(a0 + i) + d];
      mn[d] = x < mn[d] ? x : mn[d];
      mx[d] = x > mx[d] ? x : mx[d];
    }
  for (int o = 32; o >= 1; o >>= 1)
    for (int d = 0; d < 3; ++d) {
      const int a = __shfl_xor(mn[d], o, 64), b = __shfl_xor(mx[d], o, 64);
      mn[d] = a < mn[d] ? a : mn[d];
      mx[d] = b > mx[d] ? b : mx[d];
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      S.red[wave][d] = mn[d];
      S.red[wave][3 + d] = mx[d];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    int wide = 0;
    for (int d = 0; d < 3; ++d) {
      int a = S.red[0][d], b = S.red[0][3 + d];
      for (int w = 1; w < kThreads / 64; ++w) {
        a = S.red[w][d] < a ? S.red[w][d] : a;
        b = S.red[w][3 + d] > b ? S.red[w][3 + d] : b;
      }
      if (n > 0 && (int64_t)b - a >= ((int64_t)1 << 31)) wide = 1;
    }
    S.wide = wide;
  }
  __syncthreads();
  return S.wide;
}

// stages atoms j0 .. j0 + jn - 1 of the pose into the tile
__device__ inline void stage_tile(GraphShared &S, const int32_t *__restrict__ xyz, int a0, int j0, int jn) {
  for (int t = threadIdx.x; t < jn; t += kThreads) {
    const int32_t *q = xyz + 3 * (int64_t)(a0 + j0 + t);
    S.tile[t] = make_int4(q[0], q[1], q[2], 0);
  }
}

// squared distance, exact (see the header); ~0 when a wide pose's pair fails the box
template <bool WIDE>
__device__ inline unsigned long long dist2(int4 q, int xi, int yi, int zi, int r) {
  if (!WIDE) {
    const unsigned ax = (unsigned)abs(q.x - xi), ay = (unsigned)abs(q.y - yi), az = (unsigned)abs(q.z - zi);
    return (unsigned long long)ax * ax + (unsigned long long)ay * ay + (unsigned long long)az * az;
  } else {
    const long long ex = (long long)q.x - xi, ey = (long long)q.y - yi, ez = (long long)q.z - zi;
    if (ex < -r || ex > r || ey < -r || ey > r || ez < -r || ez > r) return ~0ull;
    return (unsigned long long)(ex * ex + ey * ey + ez * ez);
  }
}

// Pass 1 body: degrees of atom i (i < n) against all atoms of the pose.  Every
// thread of the workgroup calls it (the tile is shared); `act` marks a real atom.
template <bool WIDE>
__device__ inline void count_sweep(GraphShared &S, const int32_t *__restrict__ xyz, int a0, int n, int i0,
                                   int r_cov, int r_nc, int &dc, int &dn) {
  const int i = i0 + threadIdx.x;
  const bool act = i < n;
  int xi = 0, yi = 0, zi = 0;
  if (act) {
    xi = xyz[3 * (int64_t)(a0 + i)];
    yi = xyz[3 * (int64_t)(a0 + i) + 1];
    zi = xyz[3 * (int64_t)(a0 + i) + 2];
  }
  const unsigned long long rc2 = (unsigned long long)r_cov * r_cov, rn2 = (unsigned long long)r_nc * r_nc;
  int cc = 0, cn = 0;
  for (int j0 = 0; j0 < n; j0 += kTile) {
    const int jn = n - j0 < kTile ? n - j0 : kTile;
    if (!(n <= kTile && i0 > 0)) {  // one tile holding the whole pose is staged once
      __syncthreads();
      stage_tile(S, xyz, a0, j0, jn);
      __syncthreads();
    }
    if (act) {
#pragma unroll 4
      for (int jj = 0; jj < jn; ++jj) {
        const unsigned long long D = dist2<WIDE>(S.tile[jj], xi, yi, zi, r_nc);
        cn += D <= rn2;
        cc += D <= rc2;
      }
    }
  }
  dc = cc - 1;  // the atom itself (distance 0) is not an edge
  dn = cn - 1;
}

__global__ __launch_bounds__(kThreads) void k_graph_count(const int32_t *__restrict__ atom_off, int n_atoms,
                                                          const int32_t *__restrict__ xyz, int p0,
                                                          int r_cov, int r_nc,
                                                          int32_t *__restrict__ deg,  // [2][Nchunk]
                                                          int64_t n_chunk_cap,
                                                          int64_t *__restrict__ pose_tot,  // [2][P]
                                                          int n_poses, int64_t *status) {
  __shared__ GraphShared S;
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  if ((!pose_range(atom_off, p0 + pl, n_atoms, a0, a1) || a0 < base) && threadIdx.x == 0)
    dev_fail(status, kDevBadOffsets);
  if (a0 < base) a0 = a1 = base;
  int n = a1 - a0;
  if (n < 0 || n > CF_MAX_POSE_ATOMS) {
    if (threadIdx.x == 0) dev_fail(status, n < 0 ? kDevBadOffsets : kDevPoseTooLarge);
    n = 0;
  }
  const int wide = pose_is_wide(S, xyz, a0, n);
  long long tc = 0, tn = 0;
  for (int i0 = 0; i0 < n; i0 += kThreads) {
    int dc, dn;
    if (wide)
      count_sweep<true>(S, xyz, a0, n, i0, r_cov, r_nc, dc, dn);
    else
      count_sweep<false>(S, xyz, a0, n, i0, r_cov, r_nc, dc, dn);
    const int i = i0 + threadIdx.x;
    const int64_t li = (int64_t)(a0 - base) + i;
    if (i < n) {
      if (li < n_chunk_cap) {
        deg[li] = dc;
        deg[n_chunk_cap + li] = dn;
      }
      tc += dc;
      tn += dn;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    tc += __shfl_xor(tc, o, 64);
    tn += __shfl_xor(tn, o, 64);
  }
  __shared__ long long red2[kThreads / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red2[wave][0] = tc;
    red2[wave][1] = tn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long a = 0, b = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      a += red2[w][0];
      b += red2[w][1];
    }
    pose_tot[pl] = a;
    pose_tot[n_poses + pl] = b;
  }
}

// Exclusive scan of per-pose edge totals (one workgroup); writes the closing
// row_ptr entries and checks capacities.
__global__ __launch_bounds__(1024) void k_graph_scan(const int32_t *__restrict__ atom_off, int p0,
                                                     int n_poses, int64_t n_chunk_cap,
                                                     int64_t *__restrict__ pose_tot,
                                                     int32_t *cov_row, int64_t cov_cap, int32_t *nc_row,
                                                     int64_t nc_cap, int64_t *status) {
  __shared__ long long tmp[2][1024];
  long long carry[2] = {0, 0};
  for (int b0 = 0; b0 < n_poses; b0 += 1024) {
    const int p = b0 + threadIdx.x;
    for (int t = 0; t < 2; ++t) tmp[t][threadIdx.x] = p < n_poses ? pose_tot[t * n_poses + p] : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      long long v[2];
      for (int t = 0; t < 2; ++t) v[t] = threadIdx.x >= o ? tmp[t][threadIdx.x - o] : 0;
      __syncthreads();
      for (int t = 0; t < 2; ++t) tmp[t][threadIdx.x] += v[t];
      __syncthreads();
    }
    for (int t = 0; t < 2; ++t) {
      const long long incl = tmp[t][threadIdx.x];
      const long long own = p < n_poses ? pose_tot[t * n_poses + p] : 0;
      if (p < n_poses) pose_tot[(2 + t) * n_poses + p] = carry[t] + incl - own;  // exclusive offset
    }
    __syncthreads();
    for (int t = 0; t < 2; ++t) carry[t] += tmp[t][1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t nchunk = (int64_t)atom_off[p0 + n_poses] - atom_off[p0];
    const bool over = carry[0] > cov_cap || carry[1] > nc_cap || carry[0] > INT32_MAX || carry[1] > INT32_MAX;
    if (over) {
      dev_fail(status, kDevCapacity);
      atomicMax(reinterpret_cast<unsigned long long *>(status + 1), (unsigned long long)carry[0]);
      atomicMax(reinterpret_cast<unsigned long long *>(status + 2), (unsigned long long)carry[1]);
    }
    if (nchunk >= 0 && nchunk <= n_chunk_cap) {
      cov_row[nchunk] = (int32_t)(carry[0] > INT32_MAX ? INT32_MAX : carry[0]);
      nc_row[nchunk] = (int32_t)(carry[1] > INT32_MAX ? INT32_MAX : carry[1]);
    } else {
      dev_fail(status, kDevBadOffsets);
    }
  }
}

// Pass 2 body: the row of atom i, columns in ascending order.  A row is written
// only if it fits its capacity whole; sc / sn are its first slots.
template <bool WIDE>
__device__ inline void fill_sweep(GraphShared &S, const int32_t *__restrict__ xyz, int a0, int n, int i0, int lb,
                                  int r_cov, int r_nc, bool act, int64_t sc, int64_t sn, int dc, int dn, bool wc,
                                  bool wn, int32_t *cov_col, int32_t *nc_col) {
  const int i = i0 + threadIdx.x;
  int xi = 0, yi = 0, zi = 0;
  if (act) {
    xi = xyz[3 * (int64_t)(a0 + i)];
    yi = xyz[3 * (int64_t)(a0 + i) + 1];
    zi = xyz[3 * (int64_t)(a0 + i) + 2];
  }
  const unsigned long long rc2 = (unsigned long long)r_cov * r_cov, rn2 = (unsigned long long)r_nc * r_nc;
  int kc = 0, kn = 0;
  for (int j0 = 0; j0 < n; j0 += kTile) {
    const int jn = n - j0 < kTile ? n - j0 : kTile;
    if (!(n <= kTile && i0 > 0)) {
      __syncthreads();
      stage_tile(S, xyz, a0, j0, jn);
      __syncthreads();
    }
    if (act) {
#pragma unroll 2
      for (int jj = 0; jj < jn; ++jj) {
        const unsigned long long D = dist2<WIDE>(S.tile[jj], xi, yi, zi, r_nc);
        const int j = j0 + jj;
        if (D <= rn2 && j != i) {
          if (wn && kn < dn) nc_col[sn + kn] = lb + j;
          ++kn;
          if (D <= rc2) {
            if (wc && kc < dc) cov_col[sc + kc] = lb + j;
            ++kc;
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_graph_fill(const int32_t *__restrict__ atom_off, int n_atoms,
                                                         const int32_t *__restrict__ xyz, int p0,
                                                         int r_cov, int r_nc,
                                                         const int32_t *__restrict__ deg,
                                                         int64_t n_chunk_cap,
                                                         const int64_t *__restrict__ pose_tot,
                                                         int n_poses, int32_t *cov_row, int32_t *cov_col,
                                                         int64_t cov_cap, int32_t *nc_row, int32_t *nc_col,
                                                         int64_t nc_cap, int64_t *status) {
  __shared__ GraphShared S;
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  if ((!pose_range(atom_off, p0 + pl, n_atoms, a0, a1) || a0 < base) && threadIdx.x == 0)
    dev_fail(status, kDevBadOffsets);
  if (a0 < base) a0 = a1 = base;
  const int n = a1 - a0;
  if (n <= 0 || n > CF_MAX_POSE_ATOMS) return;  // reported by pass 1
  const int64_t off_c = pose_tot[2 * n_poses + pl], off_n = pose_tot[3 * n_poses + pl];
  const int lb = a0 - base;
  const int wide = pose_is_wide(S, xyz, a0, n);
  int64_t run_c = off_c, run_n = off_n;
  for (int i0 = 0; i0 < n; i0 += kThreads) {
    // row pointers: exclusive scan of this round's degrees
    const int i = i0 + threadIdx.x;
    const bool act = i < n && lb + i < n_chunk_cap;
    const int dc = act ? deg[lb + i] : 0;
    const int dn = act ? deg[n_chunk_cap + lb + i] : 0;
    int tc, tn;
    const int ec = block_excl_scan(dc, S.scan_tmp, &tc);
    const int en = block_excl_scan(dn, S.scan_tmp, &tn);
    const int64_t sc = run_c + ec, sn = run_n + en;
    if (act) {
      cov_row[lb + i] = (int32_t)(sc > INT32_MAX ? INT32_MAX : sc);
      nc_row[lb + i] = (int32_t)(sn > INT32_MAX ? INT32_MAX : sn);
    }
    run_c += tc;
    run_n += tn;
    const bool wc = sc + dc <= cov_cap, wn = sn + dn <= nc_cap;
    if (wide)
      fill_sweep<true>(S, xyz, a0, n, i0, lb, r_cov, r_nc, act, sc, sn, dc, dn, wc, wn, cov_col, nc_col);
    else
      fill_sweep<false>(S, xyz, a0, n, i0, lb, r_cov, r_nc, act, sc, sn, dc, dn, wc, wn, cov_col, nc_col);
  }
}

}  // namespace

hipError_t launch_graph(const int32_t *atom_off, int n_atoms, const int32_t *xyz, int p0, int n_poses, int r_cov,
                        int r_nc, int32_t *cov_row, int32_t *cov_col, int64_t cov_cap, int32_t *nc_row,
                        int32_t *nc_col, int64_t nc_cap, int32_t *deg_scratch, int64_t n_chunk_cap,
                        int64_t *pose_scratch, int64_t *status, hipStream_t s) {
  // deg_scratch: 2 * n_chunk_cap ints; pose_scratch: 4 * n_poses int64
  if (n_poses <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_graph_count, dim3(n_poses), dim3(kThreads), 0, s, atom_off, n_atoms, xyz, p0, r_cov,
                     r_nc, deg_scratch, n_chunk_cap, pose_scratch, n_poses, status);
  hipLaunchKernelGGL(k_graph_scan, dim3(1), dim3(1024), 0, s, atom_off, p0, n_poses, n_chunk_cap, pose_scratch,
                     cov_row, cov_cap, nc_row, nc_cap, status);
  hipLaunchKernelGGL(k_graph_fill, dim3(n_poses), dim3(kThreads), 0, s, atom_off, n_atoms, xyz, p0, r_cov,
                     r_nc, deg_scratch, n_chunk_cap, pose_scratch, n_poses, cov_row, cov_col, cov_cap,
                     nc_row, nc_col, nc_cap, status);
  return hipGetLastError();
}

}  // namespace cf
