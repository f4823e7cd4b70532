// Covalent and non-covalent neighbour lists by exact integer distance tests.
//
// The SG-CNN reads a spatial graph with two edge types chosen by distance
// threshold (Sec. 1; thresholds are hyper-parameters, Table I / Table II).  An
// edge (i, j) exists for i != j in the same pose when |x_i - x_j|^2 <= r^2 with
// coordinates and r in 2^-10 A integers, so the lists are exact.
//
// Design: one workgroup per pose.  Atom coordinates are staged in LDS and binned
// into a cell grid (cell edge >= r_nc, at most 16^3 cells) by an LDS counting
// sort; each thread then tests the 27 neighbouring cells of its atoms.  Pass 1
// counts degrees, a single-workgroup scan turns per-pose totals into edge
// offsets, and pass 2 writes every row and sorts it (rows are short), which gives
// the canonical ascending column order independent of thread timing.
#include <climits>

#include "cf_internal.h"

namespace cf {

namespace {

constexpr int kCellsPerAxis = 16;
constexpr int kNCell = kCellsPerAxis * kCellsPerAxis * kCellsPerAxis;
constexpr int kThreads = 256;

struct GraphShared {
  int xyz[CF_MAX_POSE_ATOMS][3];
  int cell_start[kNCell + 1];
  int cell_fill[kNCell];
  unsigned short sorted[CF_MAX_POSE_ATOMS];
  unsigned short cell_of[CF_MAX_POSE_ATOMS];
  long long red[kThreads / 64][6];
  int scan_tmp[kThreads];
  long long cs;
  int lo[3];
  int bad;
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

// Builds the per-pose cell list in LDS.  Returns the atom count n (or -1 when the
// pose cannot be handled, after flagging the status word).
__device__ int build_cells(GraphShared &S, const int32_t *__restrict__ xyz, int a0, int a1,
                           int r_nc, int64_t *status) {
  const int n = a1 - a0;
  if (threadIdx.x == 0) S.bad = 0;
  if (n < 0 || n > CF_MAX_POSE_ATOMS) {
    if (threadIdx.x == 0) dev_fail(status, n < 0 ? kDevBadOffsets : kDevPoseTooLarge);
    return -1;
  }
  long long mn[3] = {LLONG_MAX, LLONG_MAX, LLONG_MAX}, mx[3] = {LLONG_MIN, LLONG_MIN, LLONG_MIN};
  for (int i = threadIdx.x; i < n; i += kThreads) {
    for (int d = 0; d < 3; ++d) {
      const int x = xyz[3 * (int64_t)(a0 + i) + d];
      S.xyz[i][d] = x;
      mn[d] = x < mn[d] ? x : mn[d];
      mx[d] = x > mx[d] ? x : mx[d];
    }
  }
  for (int o = 32; o >= 1; o >>= 1)
    for (int d = 0; d < 3; ++d) {
      const long long a = __shfl_xor(mn[d], o, 64), b = __shfl_xor(mx[d], o, 64);
      mn[d] = a < mn[d] ? a : mn[d];
      mx[d] = b > mx[d] ? b : mx[d];
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      S.red[wave][d] = mn[d];
      S.red[wave][3 + d] = mx[d];
    }
  for (int c = threadIdx.x; c < kNCell; c += kThreads) S.cell_fill[c] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long ext = 0;
    for (int d = 0; d < 3; ++d) {
      long long a = S.red[0][d], b = S.red[0][3 + d];
      for (int w = 1; w < kThreads / 64; ++w) {
        a = S.red[w][d] < a ? S.red[w][d] : a;
        b = S.red[w][3 + d] > b ? S.red[w][3 + d] : b;
      }
      S.lo[d] = n > 0 ? (int)a : 0;
      if (n > 0 && b - a > ext) ext = b - a;
    }
    long long cs = ext / (kCellsPerAxis - 1) + 1;
    if (cs < r_nc) cs = r_nc;
    if (cs < 1) cs = 1;
    S.cs = cs;
  }
  __syncthreads();
  const long long cs = S.cs;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int cx = (int)((S.xyz[i][0] - (long long)S.lo[0]) / cs);
    const int cy = (int)((S.xyz[i][1] - (long long)S.lo[1]) / cs);
    const int cz = (int)((S.xyz[i][2] - (long long)S.lo[2]) / cs);
    const int c = (cx * kCellsPerAxis + cy) * kCellsPerAxis + cz;
    S.cell_of[i] = (unsigned short)c;
    atomicAdd(&S.cell_fill[c], 1);
  }
  __syncthreads();
  // exclusive scan of the cell counts: each thread owns 16 consecutive cells
  constexpr int per = kNCell / kThreads;
  int local = 0;
  for (int q = 0; q < per; ++q) local += S.cell_fill[threadIdx.x * per + q];
  int total;
  int run = block_excl_scan(local, S.scan_tmp, &total);
  for (int q = 0; q < per; ++q) {
    const int c = threadIdx.x * per + q;
    S.cell_start[c] = run;
    run += S.cell_fill[c];
    S.cell_fill[c] = 0;
  }
  if (threadIdx.x == 0) S.cell_start[kNCell] = total;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const int c = S.cell_of[i];
    const int pos = S.cell_start[c] + atomicAdd(&S.cell_fill[c], 1);
    S.sorted[pos] = (unsigned short)i;
  }
  __syncthreads();
  return n;
}

// Visits every j != i of the pose within r_nc of atom i (any order).
template <typename F>
__device__ inline void for_neighbours(const GraphShared &S, int i, long long rnc2, F &&f) {
  const int c = S.cell_of[i];
  const int cx = c / (kCellsPerAxis * kCellsPerAxis), cy = (c / kCellsPerAxis) % kCellsPerAxis,
            cz = c % kCellsPerAxis;
  const long long xi = S.xyz[i][0], yi = S.xyz[i][1], zi = S.xyz[i][2];
  for (int dx = -1; dx <= 1; ++dx) {
    const int ax = cx + dx;
    if (ax < 0 || ax >= kCellsPerAxis) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int ay = cy + dy;
      if (ay < 0 || ay >= kCellsPerAxis) continue;
      for (int dz = -1; dz <= 1; ++dz) {
        const int az = cz + dz;
        if (az < 0 || az >= kCellsPerAxis) continue;
        const int cc = (ax * kCellsPerAxis + ay) * kCellsPerAxis + az;
        for (int q = S.cell_start[cc]; q < S.cell_start[cc + 1]; ++q) {
          const int j = S.sorted[q];
          if (j == i) continue;
          const long long ex = S.xyz[j][0] - xi, ey = S.xyz[j][1] - yi, ez = S.xyz[j][2] - zi;
          const long long D = ex * ex + ey * ey + ez * ez;
          if (D <= rnc2) f(j, D);
        }
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_graph_count(const int32_t *__restrict__ atom_off, int n_atoms,
                                                          const int32_t *__restrict__ xyz, int p0,
                                                          int r_cov, int r_nc,
                                                          int32_t *__restrict__ deg,  // [2][Nchunk]
                                                          int64_t n_chunk_cap,
                                                          int64_t *__restrict__ pose_tot,  // [2][P]
                                                          int n_poses, int64_t *status) {
  extern __shared__ char smem[];
  GraphShared &S = *reinterpret_cast<GraphShared *>(smem);
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  if ((!pose_range(atom_off, p0 + pl, n_atoms, a0, a1) || a0 < base) && threadIdx.x == 0)
    dev_fail(status, kDevBadOffsets);
  if (a0 < base) a0 = a1 = base;
  const int n = build_cells(S, xyz, a0, a1, r_nc, status);
  long long tc = 0, tn = 0;
  if (n > 0) {
    const long long rc2 = (long long)r_cov * r_cov, rn2 = (long long)r_nc * r_nc;
    for (int i = threadIdx.x; i < n; i += kThreads) {
      int dc = 0, dn = 0;
      for_neighbours(S, i, rn2, [&](int, long long D) {
        dn += 1;
        dc += D <= rc2;
      });
      const int64_t li = (int64_t)(a0 - base) + i;
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
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    S.red[wave][0] = tc;
    S.red[wave][1] = tn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long a = 0, b = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      a += S.red[w][0];
      b += S.red[w][1];
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

__device__ inline void insert_sorted(int32_t *row, int k, int32_t v) {
  int q = k;
  while (q > 0 && row[q - 1] > v) {
    row[q] = row[q - 1];
    --q;
  }
  row[q] = v;
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
  extern __shared__ char smem[];
  GraphShared &S = *reinterpret_cast<GraphShared *>(smem);
  const int pl = blockIdx.x;
  const int base = atom_off[p0];
  int a0, a1;
  if ((!pose_range(atom_off, p0 + pl, n_atoms, a0, a1) || a0 < base) && threadIdx.x == 0)
    dev_fail(status, kDevBadOffsets);
  if (a0 < base) a0 = a1 = base;
  const int n = build_cells(S, xyz, a0, a1, r_nc, status);
  if (n <= 0) return;
  const int64_t off_c = pose_tot[2 * n_poses + pl], off_n = pose_tot[3 * n_poses + pl];
  const int64_t lb = (int64_t)(a0 - base);
  // row pointers: exclusive scan of degrees over the pose's atoms, in chunks of kThreads
  int64_t run_c = off_c, run_n = off_n;
  for (int i0 = 0; i0 < n; i0 += kThreads) {
    const int i = i0 + threadIdx.x;
    const int dc = (i < n && lb + i < n_chunk_cap) ? deg[lb + i] : 0;
    const int dn = (i < n && lb + i < n_chunk_cap) ? deg[n_chunk_cap + lb + i] : 0;
    int tc, tn;
    const int ec = block_excl_scan(dc, S.scan_tmp, &tc);
    const int en = block_excl_scan(dn, S.scan_tmp, &tn);
    if (i < n && lb + i < n_chunk_cap) {
      const int64_t rc = run_c + ec, rn = run_n + en;
      cov_row[lb + i] = (int32_t)(rc > INT32_MAX ? INT32_MAX : rc);
      nc_row[lb + i] = (int32_t)(rn > INT32_MAX ? INT32_MAX : rn);
    }
    run_c += tc;
    run_n += tn;
  }
  __syncthreads();
  const long long rc2 = (long long)r_cov * r_cov, rn2 = (long long)r_nc * r_nc;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    if (lb + i >= n_chunk_cap) break;
    const int64_t sc = cov_row[lb + i], sn = nc_row[lb + i];
    const int64_t dc = deg[lb + i], dn = deg[n_chunk_cap + lb + i];
    const bool wc = sc + dc <= cov_cap, wn = sn + dn <= nc_cap;
    int kc = 0, kn = 0;
    for_neighbours(S, i, rn2, [&](int j, long long D) {
      const int32_t col = (int32_t)(lb + j);
      if (wn && kn < dn) insert_sorted(nc_col + sn, kn, col);
      kn += 1;
      if (D <= rc2) {
        if (wc && kc < dc) insert_sorted(cov_col + sc, kc, col);
        kc += 1;
      }
    });
  }
}

}  // namespace

hipError_t launch_graph(const int32_t *atom_off, int n_atoms, const int32_t *xyz, int p0, int n_poses, int r_cov,
                        int r_nc, int32_t *cov_row, int32_t *cov_col, int64_t cov_cap, int32_t *nc_row,
                        int32_t *nc_col, int64_t nc_cap, int32_t *deg_scratch, int64_t n_chunk_cap,
                        int64_t *pose_scratch, int64_t *status, hipStream_t s) {
  // deg_scratch: 2 * n_chunk_cap ints; pose_scratch: 4 * n_poses int64
  if (n_poses <= 0) return hipSuccess;
  const size_t lds = sizeof(GraphShared);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graph_count), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graph_fill), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_graph_count, dim3(n_poses), dim3(kThreads), lds, s, atom_off, n_atoms, xyz, p0, r_cov,
                     r_nc, deg_scratch, n_chunk_cap, pose_scratch, n_poses, status);
  hipLaunchKernelGGL(k_graph_scan, dim3(1), dim3(1024), 0, s, atom_off, p0, n_poses, n_chunk_cap, pose_scratch,
                     cov_row, cov_cap, nc_row, nc_cap, status);
  hipLaunchKernelGGL(k_graph_fill, dim3(n_poses), dim3(kThreads), lds, s, atom_off, n_atoms, xyz, p0, r_cov,
                     r_nc, deg_scratch, n_chunk_cap, pose_scratch, n_poses, cov_row, cov_col, cov_cap,
                     nc_row, nc_col, nc_cap, status);
  return hipGetLastError();
}

}  // namespace cf
