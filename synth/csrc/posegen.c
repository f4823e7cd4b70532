/*
 * Seeded synthetic docked-pose generator (input generation only; holds none of
 * the scoring method's arithmetic).
 *
 * The paper scores docked protein-ligand poses (Sec. 4, 4.2) whose featurisation
 * it takes unchanged from its predecessor (Sec. 3.3).  No poses ship with the
 * paper, so this file builds stand-ins with the shapes of that workload:
 *   - ligand: a random branched chain; each new atom bonds to a uniformly chosen
 *     existing atom of degree < 4, along a uniform direction, at a bond length
 *     drawn from U[1.45, 1.55] A; a candidate closer than 2.0 A to any atom other
 *     than its parent is redrawn;
 *   - pocket: atoms drawn uniformly in a spherical shell [r_in, r_out] around the
 *     ligand centroid (r^3 uniform, direction uniform), redrawn when closer than
 *     2.5 A to any placed atom; after `jam` consecutive redraws the outer radius
 *     grows by 0.5 A (a shell of fixed size jams long before 900 atoms fit);
 *   - elements C .62, N .17, O .18, S .02, halogen .01 and 19 feature channels:
 *     0-10 one-hot [C,N,O,S,halogen,P,B,Se,metal,H,other], 11 hybridisation,
 *     12 heavy valence, 13 hetero valence, 14 partial charge, 15 hydrophobic,
 *     16 aromatic, 17 donor/acceptor, 18 ligand(+1)/pocket(-1) flag;
 *   - coordinates: int32 in units of 2^-10 A (round to nearest even).
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  Its i-th
 * output from state s is mix(s + (i+1)*0x9E3779B97F4A7C15), so it is counter
 * based; every pose has its own stream keyed by (seed, stream tag, pose index),
 * which makes a pose bit-identical whether it is generated alone or in a batch.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NCH 19
#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

typedef struct { uint64_t s; } rng_t;

static inline uint64_t rnext(rng_t *r) { r->s += GOLDEN; return mix64(r->s); }
/* uniform double in [0,1) from the top 53 bits */
static inline double runif(rng_t *r) { return (double)(rnext(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [lo, hi] (inclusive); modulo bias < 2^-40 for these ranges */
static inline int rint_range(rng_t *r, int lo, int hi) {
  return lo + (int)(rnext(r) % (uint64_t)(hi - lo + 1));
}
/* standard normal by the Box-Muller transform (one value per call) */
static double rnorm(rng_t *r) {
  double u1 = runif(r), u2 = runif(r);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
static void rdir(rng_t *r, double d[3]) {
  double z = 2.0 * runif(r) - 1.0, phi = 6.283185307179586 * runif(r);
  double s = sqrt(fmax(0.0, 1.0 - z * z));
  d[0] = s * cos(phi); d[1] = s * sin(phi); d[2] = z;
}

uint64_t cfgen_pose_key(uint64_t seed, uint64_t stream, uint64_t pose) {
  return mix64(mix64(seed * GOLDEN + stream) + (pose + 1) * GOLDEN);
}

/* ---- spatial hash for the rejection tests (cell 2.5 A, dense 96^3 window) ---- */
#define HC 96
#define HCELL 2.5
typedef struct {
  int *head;   /* [HC^3] */
  int *next;   /* [cap] */
  double org;  /* window origin (same on every axis) */
} hash_t;

static int hcell(const hash_t *h, const double p[3], int c[3]) {
  for (int a = 0; a < 3; ++a) {
    int i = (int)floor((p[a] - h->org) / HCELL);
    if (i < 0 || i >= HC) return -1;
    c[a] = i;
  }
  return (c[0] * HC + c[1]) * HC + c[2];
}

static void hinsert(hash_t *h, const double *pos, int idx) {
  int c[3];
  int k = hcell(h, pos + 3 * idx, c);
  if (k < 0) return; /* never happens for the radii used (window is 240 A) */
  h->next[idx] = h->head[k];
  h->head[k] = idx;
}

/* 1 if p is at least rmin from every inserted atom except `skip` */
static int hclear(const hash_t *h, const double *pos, const double p[3], double rmin, int skip) {
  int c[3];
  if (hcell(h, p, c) < 0) return 0;
  double r2 = rmin * rmin;
  int reach = (int)ceil(rmin / HCELL);
  for (int a = c[0] - reach; a <= c[0] + reach; ++a) {
    if (a < 0 || a >= HC) continue;
    for (int b = c[1] - reach; b <= c[1] + reach; ++b) {
      if (b < 0 || b >= HC) continue;
      for (int d = c[2] - reach; d <= c[2] + reach; ++d) {
        if (d < 0 || d >= HC) continue;
        for (int j = h->head[(a * HC + b) * HC + d]; j >= 0; j = h->next[j]) {
          if (j == skip) continue;
          double dx = p[0] - pos[3 * j], dy = p[1] - pos[3 * j + 1], dz = p[2] - pos[3 * j + 2];
          if (dx * dx + dy * dy + dz * dz < r2) return 0;
        }
      }
    }
  }
  return 1;
}

/* element classes: 0 C, 1 N, 2 O, 3 S, 4 halogen */
static int draw_element(rng_t *r) {
  double u = runif(r);
  if (u < 0.62) return 0;
  if (u < 0.79) return 1;
  if (u < 0.97) return 2;
  if (u < 0.99) return 3;
  return 4;
}

/*
 * Atom-count draw for one pose.  mode 0: n_lig ~ U{lig_lo..lig_hi},
 * n_pocket ~ U{pock_lo..pock_hi}.  mode 1: total ~ log-uniform [tot_lo, tot_hi]
 * (rounded to nearest), n_lig ~ U{20 .. min(60, total/5)}, n_pocket = total - n_lig.
 */
void cfgen_pose_sizes(uint64_t seed, uint64_t stream, int64_t pose0, int64_t n_poses, int mode,
                      const int32_t *lim, int32_t *n_lig_out, int32_t *n_pock_out) {
  for (int64_t p = 0; p < n_poses; ++p) {
    rng_t r = {cfgen_pose_key(seed, stream ^ 0x51CE5ULL, (uint64_t)(pose0 + p))};
    if (mode == 0) {
      n_lig_out[p] = rint_range(&r, lim[0], lim[1]);
      n_pock_out[p] = rint_range(&r, lim[2], lim[3]);
    } else {
      double lo = log((double)lim[0]), hi = log((double)lim[1]);
      int tot = (int)llrint(exp(lo + (hi - lo) * runif(&r)));
      if (tot < lim[0]) tot = lim[0];
      if (tot > lim[1]) tot = lim[1];
      int lig_hi = tot / 5 < 60 ? tot / 5 : 60;
      if (lig_hi < 20) lig_hi = 20;
      n_lig_out[p] = rint_range(&r, 20, lig_hi);
      n_pock_out[p] = tot - n_lig_out[p];
    }
  }
}

/*
 * Generate one pose with n_lig ligand atoms followed by n_pock pocket atoms.
 * Writes xyz [n][3] (int32, 2^-10 A), feat [n][19] (f32), is_lig [n] (u8).
 * `work` must hold 3*(n) doubles + HC^3 + n ints (see cfgen_work_bytes).
 * Returns the final outer shell radius in A (diagnostic), or -1 on failure.
 */
size_t cfgen_work_bytes(int n) {
  return sizeof(double) * 3 * (size_t)n + sizeof(int) * ((size_t)HC * HC * HC + (size_t)n + 8 * (size_t)n);
}

double cfgen_pose(uint64_t seed, uint64_t stream, int64_t pose, int n_lig, int n_pock,
                  double r_in, double r_out, int jam, void *work,
                  int32_t *xyz, float *feat, uint8_t *is_lig) {
  int n = n_lig + n_pock;
  rng_t r = {cfgen_pose_key(seed, stream, (uint64_t)pose)};
  double *pos = (double *)work;
  hash_t h;
  h.head = (int *)(pos + 3 * (size_t)n);
  h.next = h.head + (size_t)HC * HC * HC;
  int *deg = h.next + n;        /* ligand covalent degree */
  int *nbr = deg + n;           /* up to 4 bonded neighbours per ligand atom */
  int *elem = nbr + 4 * (size_t)n;
  int *cand = elem + n;         /* candidate parents */
  for (size_t i = 0; i < (size_t)HC * HC * HC; ++i) h.head[i] = -1;
  h.org = -HC * HCELL / 2.0;
  memset(deg, 0, sizeof(int) * n);

  /* ligand chain */
  pos[0] = pos[1] = pos[2] = 0.0;
  hinsert(&h, pos, 0);
  for (int a = 1; a < n_lig; ++a) {
    int placed = 0;
    for (int tries = 0; tries < 100000 && !placed; ++tries) {
      int nc = 0;
      for (int j = 0; j < a; ++j)
        if (deg[j] < 4) cand[nc++] = j;
      if (nc == 0) return -1.0;
      int par = cand[rint_range(&r, 0, nc - 1)];
      double d[3];
      rdir(&r, d);
      double len = 1.45 + 0.10 * runif(&r);
      double p[3] = {pos[3 * par] + len * d[0], pos[3 * par + 1] + len * d[1], pos[3 * par + 2] + len * d[2]};
      if (!hclear(&h, pos, p, 2.0, par)) continue;
      pos[3 * a] = p[0]; pos[3 * a + 1] = p[1]; pos[3 * a + 2] = p[2];
      hinsert(&h, pos, a);
      nbr[4 * par + deg[par]] = a; deg[par]++;
      nbr[4 * a + deg[a]] = par; deg[a]++;
      placed = 1;
    }
    if (!placed) return -1.0;
  }
  double cen[3] = {0, 0, 0};
  for (int a = 0; a < n_lig; ++a)
    for (int k = 0; k < 3; ++k) cen[k] += pos[3 * a + k];
  for (int k = 0; k < 3; ++k) cen[k] /= (double)n_lig;

  /* pocket shell */
  double ro = r_out;
  for (int a = n_lig; a < n; ++a) {
    int miss = 0;
    for (;;) {
      double u = runif(&r);
      double rr = cbrt(r_in * r_in * r_in + u * (ro * ro * ro - r_in * r_in * r_in));
      double d[3];
      rdir(&r, d);
      double p[3] = {cen[0] + rr * d[0], cen[1] + rr * d[1], cen[2] + rr * d[2]};
      if (hclear(&h, pos, p, 2.5, -1)) {
        pos[3 * a] = p[0]; pos[3 * a + 1] = p[1]; pos[3 * a + 2] = p[2];
        hinsert(&h, pos, a);
        break;
      }
      if (++miss >= jam) { ro += 0.5; miss = 0; }
    }
  }

  /* elements, then features (ligand valences need every element first) */
  for (int a = 0; a < n; ++a) elem[a] = draw_element(&r);
  for (int a = 0; a < n; ++a) {
    float *f = feat + (size_t)NCH * a;
    for (int c = 0; c < NCH; ++c) f[c] = 0.0f;
    int e = elem[a];
    int lig = a < n_lig;
    f[e] = 1.0f;                                   /* one-hot slots 0-4; 5-10 stay 0 */
    f[11] = (float)rint_range(&r, 1, 3);           /* hybridisation */
    if (lig) {
      int het = 0;
      for (int b = 0; b < deg[a]; ++b) het += elem[nbr[4 * a + b]] != 0;
      f[12] = (float)deg[a];
      f[13] = (float)het;
    } else {
      f[12] = (float)rint_range(&r, 1, 3);
      f[13] = (float)rint_range(&r, 0, 2);
    }
    double q = 0.3 * rnorm(&r);
    if (q > 1.0) q = 1.0;
    if (q < -1.0) q = -1.0;
    f[14] = (float)q;
    double u15 = runif(&r), u16 = runif(&r), u17 = runif(&r);
    f[15] = (e == 0 || e == 3 || e == 4) && u15 < 0.5 ? 1.0f : 0.0f;
    f[16] = (e == 0 || e == 1) && u16 < 0.3 ? 1.0f : 0.0f;
    f[17] = (e == 1 || e == 2) && u17 < 0.6 ? 1.0f : 0.0f;
    f[18] = lig ? 1.0f : -1.0f;
    is_lig[a] = (uint8_t)lig;
  }
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < 3; ++k) {
      double v = nearbyint(pos[3 * a + k] * 1024.0); /* default rounding: nearest even */
      xyz[3 * a + k] = (int32_t)v;
    }
  return ro;
}
