// Particle kernels: drift + fixed-point CIC deposit, CIC interpolation of the
// finite-difference force + kick + drift (+ lightcone test), and the stable
// stream compaction that eliminates particles outside the lightcone.
//
// CIC (Sec. 2.4, same weights both ways for momentum conservation): the
// coordinate U = floor(x s), s = ng 2^B / L, gives the lower cell U >> B and
// the fraction q = U mod 2^B; the axis weights are (2^B - q, q) and the
// 8 products (<= 2^(3B)) are added to 64-bit integer counts, so the deposit
// is exact and independent of the order in which atomics land.
// TSC (Sec. 2.4 names it beside CIC; sdpm_config.assignment): the nearest
// node i = (U + 2^(B-1)) >> B, the offset D = U - i 2^B, and the weights of
// nodes i - 1, i, i + 1: (2^(B-1) -+ D)^2 / 2^(B+1) rounded to the nearest
// integer for the outer two and 2^B minus both for the middle, so that the
// 27 products again sum to 2^(3B) exactly.
// Leapfrog (Sec. 2.2 Eqs. 7-9): x += p (dtau/2)/a ; p += a_half g dtau ;
// x += p (dtau/2)/a_next, with g = -grad Phi by central differences.
#include "internal.h"

namespace sdpm {
namespace {

// The S x S x S mesh nodes a particle is assigned to (S = 2: CIC, S = 3:
// TSC): the first node per axis (unwrapped: it may be -1 or reach ng on a
// periodic mesh, where the users wrap it with & (ng - 1)) and, per axis, the
// fixed-point offset the weights follow from: q = U mod 2^B for CIC, D = U -
// i 2^B (i the nearest node) for TSC.
struct Frac {
  int cell[3];
  int f[3];
};
template <int S>
struct Stencil {
  int cell[3];
  uint64_t w[3][S];
};

// Axis weights in units of 2^-B from the offset f: CIC (2^B - q, q); TSC the
// nodes i - 1, i, i + 1: (2^(B-1) -+ D)^2 / 2^(B+1) rounded to the nearest
// integer for the outer two, 2^B minus both for the middle (sum exactly 2^B).
template <int S>
__device__ inline void axis_weights(int f, int frac_bits, uint64_t w[S]) {
  const uint64_t one = 1ull << frac_bits;
  if constexpr (S == 2) {
    w[0] = one - (uint64_t)f;
    w[1] = (uint64_t)f;
  } else {
    const int64_t half = (int64_t)one >> 1, D = f;
    const uint64_t wm = (uint64_t)((half - D) * (half - D) + (int64_t)one) >> (frac_bits + 1);
    const uint64_t wp = (uint64_t)((half + D) * (half + D) + (int64_t)one) >> (frac_bits + 1);
    w[0] = wm;
    w[1] = one - wm - wp;
    w[2] = wp;
  }
}

// Fixed-point coordinates of one particle.  Returns 0 or a kFlag* bit (then
// cell and offset are placeholders that no caller uses).
template <int S>
__device__ inline uint32_t assign_frac(const double x[3], const MeshMap& mm, Frac& c) {
  const int64_t span = (int64_t)mm.ng << mm.frac_bits;
  const int64_t one = 1ll << mm.frac_bits;
  uint32_t bad = 0;
  for (int d = 0; d < 3; ++d) {
    const double u = x[d] * mm.scale;
    const bool nan_or_inf = u != u || __builtin_isinf(u);
    if (nan_or_inf || !(u >= 0.0 && u <= (double)span)) {
      bad |= nan_or_inf ? kFlagOverflow : kFlagDomain;
      c.cell[d] = 0;
      c.f[d] = 0;
      continue;
    }
    int64_t U = (int64_t)floor(u);
    if (mm.periodic) U &= span - 1;
    if constexpr (S == 2) {
      c.cell[d] = (int)(U >> mm.frac_bits);
      c.f[d] = (int)(U & (one - 1));
    } else {
      const int64_t node = (U + (one >> 1)) >> mm.frac_bits;
      c.cell[d] = (int)node - 1;
      c.f[d] = (int)(U - (node << mm.frac_bits));
    }
    if (!mm.periodic && (c.cell[d] < mm.active.lo[d] || c.cell[d] + S - 1 > mm.active.hi[d]))
      bad |= kFlagDomain;
  }
  return bad;
}

// The same with the weights expanded.
template <int S>
__device__ inline uint32_t assign_setup(const double x[3], const MeshMap& mm, Stencil<S>& c) {
  Frac fr;
  const uint32_t bad = assign_frac<S>(x, mm, fr);
  for (int d = 0; d < 3; ++d) {
    c.cell[d] = fr.cell[d];
    axis_weights<S>(fr.f[d], mm.frac_bits, c.w[d]);
  }
  return bad;
}

// Position update x + p c as two roundings (no fused multiply-add), the
// leapfrog drift of Eqs. 7 and 9 as written, so that drifted positions (and
// the fixed-point cells derived from them) are the same FP64 values as those
// of a plain evaluation of the formula.
__device__ inline double drift_nofma(double x, double p, double c) {
#pragma clang fp contract(off)
  const double dp = p * c;
  return x + dp;
}

// Drift with the periodic wrap into [0, L) (a drift is far below L).
__device__ inline double drift_wrap(double x, double p, double c, const MeshMap& mm) {
  double v = drift_nofma(x, p, c);
  if (mm.periodic) {
    if (v < 0.0) v += mm.box;
    if (v >= mm.box) v -= mm.box;
  }
  return v;
}

// Squared distance ((dx^2 + dy^2) + dz^2) without fused multiply-adds, so
// that the lightcone test is the same FP64 expression everywhere.
__device__ inline double dist2_nofma(double x0, double x1, double x2, double o0, double o1,
                                     double o2) {
#pragma clang fp contract(off)
  const double dx = x0 - o0, dy = x1 - o1, dz = x2 - o2;
  const double a = dx * dx;
  const double b = dy * dy;
  const double c = dz * dz;
  return (a + b) + c;
}

// Deposit at the drifted positions (computed here, not stored),
// kDepThreads x kDepPer particles per workgroup, with the
// weights summed in LDS windows (at most kDepTile cells together) and each
// nonzero window cell added to the mesh with one global 64-bit atomic.
// Every particle is routed on its own: one whose S^3 support lies inside its
// window goes to LDS, any other (an outlier) straight to global atomics, so
// a few stray particles never push a whole workgroup onto global atomics.
// Cells are taken relative to a reference cell (thread 0's first valid
// particle; on a periodic mesh offsets wrap into [-ng/2, ng/2)).  One window
// is the workgroup's bounding box when that fits the tile.  Otherwise (a
// workgroup of re-sorted particles that straddles two blocks, which need
// not be neighbours along every axis) the particles split in two groups at
// the first particle in memory order that lies in the last particle's
// block, each group with its own window: its bounding box if both fit, else
// boxes of a share of the tile centred on the group's mean offset, the axes
// with the smallest extent kept whole first; only those workgroups pay for
// the split's two further reductions.  Integer sums: the result is
// exact and the same in any order and for any routing.
constexpr int kDepThreads = 512, kDepPer = 2;
constexpr int kDepTile = 4096;       // 32 KB

__device__ inline int wave_min(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline int wave_sum(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Window of at most cap cells for the cnt particles with offsets in [mn, mx]
// (sums sm per axis), support S: the bounding box when it fits; else a box
// of at most cap cells (the axes with the smallest extent kept whole first)
// centred on the mean.  Returns its volume.
template <int S>
__device__ inline int dep_window(const int mn[3], const int mx[3], const int sm[3], int cnt,
                                 int cap, int lo[3], int w[3]) {
  int ext[3];
  double mean[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = mx[d] - mn[d] + S;
    lo[d] = mn[d];
    w[d] = ext[d];
    mean[d] = (double)sm[d] / cnt;
  }
  if ((int64_t)ext[0] * ext[1] * ext[2] <= cap) return ext[0] * ext[1] * ext[2];
  int k = 1;
  while ((k + 1) * (k + 1) * (k + 1) <= cap) ++k;
#pragma unroll
  for (int d = 0; d < 3; ++d) w[d] = min(ext[d], k);
  // rank of each axis by extent (ties in axis order); the loops below use
  // constant indices only, so that w and ext stay in registers
  int rank[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rank[d] = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e)
      if (e != d && (ext[e] < ext[d] || (ext[e] == ext[d] && e < d))) ++rank[d];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (rank[d] == r) {
        const int other = w[(d + 1) % 3] * w[(d + 2) % 3];
        w[d] = max(w[d], min(ext[d], cap / other));
      }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int start = (int)floor(mean[d] - 0.5 * (w[d] - S));
    lo[d] = min(max(start, mn[d]), mx[d] + S - w[d]);
  }
  return w[0] * w[1] * w[2];
}

// Bounding box (min, max, sum of offsets, count) of the particles a lane
// selects, reduced over the workgroup into the shared slots.
__device__ inline void dep_reduce(const int mn[3], const int mx[3], const int sm[3], int cnt,
                                  int* s_mn, int* s_mx, int* s_sum, int* s_cnt) {
  const bool lead = (threadIdx.x & 63) == 0;
  for (int d = 0; d < 3; ++d) {
    const int a = wave_min(mn[d]), b = wave_max(mx[d]), t = wave_sum(sm[d]);
    if (lead) {
      atomicMin(s_mn + d, a);
      atomicMax(s_mx + d, b);
      atomicAdd(s_sum + d, t);
    }
  }
  const int t = wave_sum(cnt);
  if (lead && t) atomicAdd(s_cnt, t);
}

template <typename PT, bool DRIFT, int S>
__global__ void __launch_bounds__(kDepThreads)
k_drift_deposit(ParticleArgs pa, double coef, MeshMap mm, unsigned long long* __restrict__ counts,
                uint32_t* __restrict__ flags) {
  __shared__ unsigned long long acc[kDepTile];
  // [0..2] reference cell (thread 0's first valid particle), [3..5] the
  // re-sort block of the last valid particle, [6] whether there is one
  __shared__ int s_ref[7];
  __shared__ int s_split;
  // [0]: all particles; [1], [2]: the two groups (only when [0] overflows)
  __shared__ int s_mn[3][3], s_mx[3][3], s_sum[3][3], s_cnt[3];
  const int tid = threadIdx.x;
  const int64_t base = xcd_block() * (kDepThreads * kDepPer);
  for (int q = tid; q < kDepTile; q += kDepThreads) acc[q] = 0ull;
  if (tid < 9) {
    s_mn[tid / 3][tid % 3] = 0x7fffffff;
    s_mx[tid / 3][tid % 3] = -0x7fffffff;
    s_sum[tid / 3][tid % 3] = 0;
  }
  if (tid < 3) s_cnt[tid] = 0;
  Frac c[kDepPer];
  bool ok[kDepPer];
  uint32_t bad_all = 0;
#pragma unroll
  for (int u = 0; u < kDepPer; ++u) {
    const int64_t i = base + u * kDepThreads + tid;
    ok[u] = false;
    if (i >= pa.n) continue;
    double x[3];
    for (int d = 0; d < 3; ++d) {
      double v = __builtin_nontemporal_load(pa.x[d] + i);
      // the drifted position is used here and not stored: the interpolation
      // pass of the step evaluates the same expression again and stores the
      // step's final position
      if (DRIFT) v = drift_wrap(v, (double)__builtin_nontemporal_load((const PT*)pa.p[d] + i), coef, mm);
      x[d] = v;
    }
    const uint32_t bad = assign_frac<S>(x, mm, c[u]);
    if (bad) {
      bad_all |= bad;
      continue;
    }
    ok[u] = true;
  }
  if (bad_all) atomicOr(flags, bad_all);
  // the reference cell (the first valid particle of thread 0) and the block
  // of the last valid particle of the last thread (the workgroup's two ends
  // in memory order), chosen by constant indices (a runtime index into c[]
  // would put it in scratch memory)
  if (tid == 0 || tid == kDepThreads - 1) {
    const bool last = tid != 0;
    int r[3] = {0, 0, 0};
    bool any = false;
#pragma unroll
    for (int q = 0; q < kDepPer; ++q) {
      // thread 0 ends on its first valid particle, the last thread on its last
      const int u = last ? q : kDepPer - 1 - q;
      if (ok[u]) {
        any = true;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          r[d] = last ? (c[u].cell[d] + (S == 3 && c[u].f[d] >= 0 ? 1 : 0)) >> mm.block_shift
                      : c[u].cell[d];
      }
    }
    if (last) {
      s_ref[3] = r[0];
      s_ref[4] = r[1];
      s_ref[5] = r[2];
      s_ref[6] = any ? 1 : 0;
    } else {
      s_ref[0] = r[0];
      s_ref[1] = r[1];
      s_ref[2] = r[2];
      s_split = 0x7fffffff;
    }
  }
  __syncthreads();
  const int ref[3] = {s_ref[0], s_ref[1], s_ref[2]};
  const int m = mm.ng - 1, half = mm.ng >> 1;
  // from here on c[u].cell holds the offset from ref
  {
    int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
    int sm[3] = {0, 0, 0};
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < kDepPer; ++u) {
      if (!ok[u]) continue;
      ++cnt;
      for (int d = 0; d < 3; ++d) {
        int o = c[u].cell[d] - ref[d];
        if (mm.periodic) o = ((o + half) & m) - half;
        c[u].cell[d] = o;
        mn[d] = min(mn[d], o);
        mx[d] = max(mx[d], o);
        sm[d] += o;
      }
    }
    dep_reduce(mn, mx, sm, cnt, s_mn[0], s_mx[0], s_sum[0], s_cnt);
  }
  __syncthreads();
  const int total = s_cnt[0];
  if (total == 0) return;                      // no valid particle in the workgroup
  // the windows (the second empty when one window takes every particle),
  // kept in separately named registers: a window chosen per particle by a
  // runtime index would put them in scratch memory
  int lo0[3], w0[3], lo1[3] = {0, 0, 0}, w1[3] = {S, S, S};
  int vol0 = 0, vol1 = 0;
  bool grp[kDepPer];
#pragma unroll
  for (int u = 0; u < kDepPer; ++u) grp[u] = false;
  const int64_t uvol = (int64_t)(s_mx[0][0] - s_mn[0][0] + S) * (s_mx[0][1] - s_mn[0][1] + S) *
                       (s_mx[0][2] - s_mn[0][2] + S);
  if (uvol <= kDepTile) {
    for (int d = 0; d < 3; ++d) {
      lo0[d] = s_mn[0][d];
      w0[d] = s_mx[0][d] - s_mn[0][d] + S;
    }
    vol0 = (int)uvol;
  } else {
    // rare: the particles split in two groups at the first particle (in
    // memory order) that lies in the last particle's re-sort block: a
    // workgroup of sorted particles straddles at most two blocks, the first
    // rows of the second following the last rows of the first; particles
    // that drifted over the shared face since the sort stay next to the group
    // they join.  Then the two groups' boxes (a uniform branch: every thread
    // read the same shared values)
    int split = 0x7fffffff;
#pragma unroll
    for (int u = 0; u < kDepPer; ++u) {
      if (!ok[u] || !s_ref[6]) continue;
      bool inb = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int home = ref[d] + c[u].cell[d] + (S == 3 && c[u].f[d] >= 0 ? 1 : 0);
        if (mm.periodic) home &= m;
        inb = inb && (home >> mm.block_shift) == s_ref[3 + d];
      }
      if (inb) split = min(split, u * kDepThreads + tid);
    }
    split = wave_min(split);
    if ((tid & 63) == 0) atomicMin(&s_split, split);
    __syncthreads();
    split = s_split;
    int mn[2][3], mx[2][3], sm[2][3], cnt[2] = {0, 0};
    for (int g = 0; g < 2; ++g)
      for (int d = 0; d < 3; ++d) {
        mn[g][d] = 0x7fffffff;
        mx[g][d] = -0x7fffffff;
        sm[g][d] = 0;
      }
#pragma unroll
    for (int u = 0; u < kDepPer; ++u) {
      if (!ok[u]) continue;
      const bool same = u * kDepThreads + tid < split;
      grp[u] = !same;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int o = c[u].cell[d];
        if (same) {
          mn[0][d] = min(mn[0][d], o);
          mx[0][d] = max(mx[0][d], o);
          sm[0][d] += o;
        } else {
          mn[1][d] = min(mn[1][d], o);
          mx[1][d] = max(mx[1][d], o);
          sm[1][d] += o;
        }
      }
      if (same) ++cnt[0]; else ++cnt[1];
    }
    dep_reduce(mn[0], mx[0], sm[0], cnt[0], s_mn[1], s_mx[1], s_sum[1], s_cnt + 1);
    dep_reduce(mn[1], mx[1], sm[1], cnt[1], s_mn[2], s_mx[2], s_sum[2], s_cnt + 2);
    __syncthreads();
    const int n0 = s_cnt[1], n1 = s_cnt[2];
    if (n0 == 0 || n1 == 0) {
      // one group only: one window of tile size over all particles
      const int g = n0 ? 1 : 2;
      vol0 = dep_window<S>(s_mn[g], s_mx[g], s_sum[g], n0 + n1, kDepTile, lo0, w0);
#pragma unroll
      for (int u = 0; u < kDepPer; ++u) grp[u] = false;
    } else {
      int64_t need[2];
      for (int g = 0; g < 2; ++g)
        need[g] = (int64_t)(s_mx[g + 1][0] - s_mn[g + 1][0] + S) *
                  (s_mx[g + 1][1] - s_mn[g + 1][1] + S) * (s_mx[g + 1][2] - s_mn[g + 1][2] + S);
      int cap0 = kDepTile / 2, cap1 = kDepTile / 2;
      if (need[0] + need[1] <= kDepTile) {
        cap0 = (int)need[0];
        cap1 = (int)need[1];
      } else if (need[1] <= kDepTile / 2) {
        cap1 = (int)need[1];
        cap0 = kDepTile - cap1;
      } else if (need[0] <= kDepTile / 2) {
        cap0 = (int)need[0];
        cap1 = kDepTile - cap0;
      }
      vol0 = dep_window<S>(s_mn[1], s_mx[1], s_sum[1], n0, cap0, lo0, w0);
      vol1 = dep_window<S>(s_mn[2], s_mx[2], s_sum[2], n1, cap1, lo1, w1);
    }
  }
#pragma unroll
  for (int u = 0; u < kDepPer; ++u) {
    if (!ok[u]) continue;
    uint64_t wt[3][S];
    for (int d = 0; d < 3; ++d) axis_weights<S>(c[u].f[d], mm.frac_bits, wt[d]);
    const bool second = grp[u];
    const int wx = second ? w1[0] : w0[0], wy = second ? w1[1] : w0[1], wz = second ? w1[2] : w0[2];
    const int r0 = c[u].cell[0] - (second ? lo1[0] : lo0[0]);
    const int r1 = c[u].cell[1] - (second ? lo1[1] : lo0[1]);
    const int r2 = c[u].cell[2] - (second ? lo1[2] : lo0[2]);
    const bool in = (unsigned)r0 <= (unsigned)(wx - S) && (unsigned)r1 <= (unsigned)(wy - S) &&
                    (unsigned)r2 <= (unsigned)(wz - S);
    if (in) {
      unsigned long long* tile = acc + (second ? vol0 : 0);
      for (int dz = 0; dz < S; ++dz)
        for (int dy = 0; dy < S; ++dy) {
          const uint64_t wyz = wt[1][dy] * wt[2][dz];
          if (wyz == 0) continue;
          const int row = ((r2 + dz) * wy + r1 + dy) * wx + r0;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = wt[0][dx] * wyz;
            if (wgt) atomicAdd(&tile[row + dx], (unsigned long long)wgt);
          }
        }
    } else {
      for (int dz = 0; dz < S; ++dz) {
        int kk = ref[2] + c[u].cell[2] + dz;
        if (mm.periodic) kk &= m;
        for (int dy = 0; dy < S; ++dy) {
          int jj = ref[1] + c[u].cell[1] + dy;
          if (mm.periodic) jj &= m;
          const uint64_t wyz = wt[1][dy] * wt[2][dz];
          if (wyz == 0) continue;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = wt[0][dx] * wyz;
            if (wgt == 0) continue;
            int ii = ref[0] + c[u].cell[0] + dx;
            if (mm.periodic) ii &= m;
            atomicAdd(counts + lin(ii, jj, kk, mm.ng), (unsigned long long)wgt);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int q = tid; q < vol0 + vol1; q += kDepThreads) {
    const unsigned long long v = acc[q];
    if (!v) continue;
    const bool second = q >= vol0;
    const int r = second ? q - vol0 : q;
    const int wx = second ? w1[0] : w0[0], wy = second ? w1[1] : w0[1];
    int gx = ref[0] + (second ? lo1[0] : lo0[0]) + r % wx;
    int gy = ref[1] + (second ? lo1[1] : lo0[1]) + (r / wx) % wy;
    int gz = ref[2] + (second ? lo1[2] : lo0[2]) + r / (wx * wy);
    if (mm.periodic) {
      gx &= m;
      gy &= m;
      gz &= m;
    }
    atomicAdd(counts + lin(gx, gy, gz, mm.ng), v);
  }
}

// g = sum over the S^3 assignment nodes of w * (-grad Phi) (central differences).
template <int S>
__device__ inline void interp_g(const double* __restrict__ phi, const MeshMap& mm,
                                const Stencil<S>& c, double inv2h, double g[3]) {
  const int n = mm.ng, m = n - 1;
  const double norm = ldexp(1.0, -3 * mm.frac_bits);
  g[0] = g[1] = g[2] = 0.0;
  for (int dz = 0; dz < S; ++dz) {
    const int k = (c.cell[2] + dz) & m;
    const int kp = (k + 1) & m, km = (k - 1) & m;
    for (int dy = 0; dy < S; ++dy) {
      const int j = (c.cell[1] + dy) & m;
      const int jp = (j + 1) & m, jm = (j - 1) & m;
      const uint64_t wyz = c.w[1][dy] * c.w[2][dz];
      for (int dx = 0; dx < S; ++dx) {
        const uint64_t wgt = c.w[0][dx] * wyz;
        const int i = (c.cell[0] + dx) & m;
        const double wd = (double)wgt * norm;
        const double gx = -(phi[lin((i + 1) & m, j, k, n)] - phi[lin((i - 1) & m, j, k, n)]) * inv2h;
        const double gy = -(phi[lin(i, jp, k, n)] - phi[lin(i, jm, k, n)]) * inv2h;
        const double gz = -(phi[lin(i, j, kp, n)] - phi[lin(i, j, km, n)]) * inv2h;
        g[0] += wd * gx;
        g[1] += wd * gy;
        g[2] += wd * gz;
      }
    }
  }
}

// The same from the FP32 force mesh g3 (3 values per cell): one 12-byte
// load per node instead of six FP64 potential values.
// Both read all S^3 nodes, zero weights included (a particle that passed
// assign_setup has them on the written mesh, so a zero weight adds an exact
// 0): without a branch per node the loads of all nodes are in flight at
// once, which measured 2.95 -> 2.28 ms for the 512^3 CIC interpolation pass.
template <int S>
__device__ inline void interp_g3(const float* __restrict__ g3, const MeshMap& mm,
                                 const Stencil<S>& c, double g[3]) {
  const int n = mm.ng, m = n - 1;
  const double norm = ldexp(1.0, -3 * mm.frac_bits);
  g[0] = g[1] = g[2] = 0.0;
  for (int dz = 0; dz < S; ++dz) {
    const int k = (c.cell[2] + dz) & m;
    for (int dy = 0; dy < S; ++dy) {
      const int j = (c.cell[1] + dy) & m;
      const uint64_t wyz = c.w[1][dy] * c.w[2][dz];
      for (int dx = 0; dx < S; ++dx) {
        const uint64_t wgt = c.w[0][dx] * wyz;
        const float* q = g3 + 3 * lin((c.cell[0] + dx) & m, j, k, n);
        const double wd = (double)wgt * norm;
        g[0] += wd * (double)q[0];
        g[1] += wd * (double)q[1];
        g[2] += wd * (double)q[2];
      }
    }
  }
}

// One particle per thread: the step's first drift by drift0_coef p (Eq. 7;
// the deposit used these positions without storing them), the force
// interpolated there, the kick with kick_coef (Eq. 8) and the second drift
// by drift_coef p (Eq. 9); only the final momenta and positions are stored.
template <typename PT, bool G3, int S>
__global__ void __launch_bounds__(256)
k_interp_kick_drift(ParticleArgs pa, const double* __restrict__ phi, const float* __restrict__ g3,
                    MeshMap mm, double inv2h, double drift0_coef,
                    double kick_coef, double drift_coef, double o0, double o1, double o2,
                    double r2, int count_removed, uint32_t* __restrict__ removed_count,
                    uint32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool out = false;
  if (i < pa.n) {
    double x[3] = {__builtin_nontemporal_load(pa.x[0] + i), __builtin_nontemporal_load(pa.x[1] + i),
                   __builtin_nontemporal_load(pa.x[2] + i)};
    // the momenta are loaded with the positions, ahead of the gathers
    const PT p_old[3] = {__builtin_nontemporal_load((const PT*)pa.p[0] + i),
                         __builtin_nontemporal_load((const PT*)pa.p[1] + i),
                         __builtin_nontemporal_load((const PT*)pa.p[2] + i)};
    // the step's first drift (Eq. 7), the same expression the deposit used
    for (int d = 0; d < 3; ++d) x[d] = drift_wrap(x[d], (double)p_old[d], drift0_coef, mm);
    Stencil<S> c;
    const uint32_t bad = assign_setup<S>(x, mm, c);
    if (bad) {
      // outside the mesh: the particle keeps the first drift only
      atomicOr(flags, bad);
      for (int d = 0; d < 3; ++d) __builtin_nontemporal_store(x[d], pa.x[d] + i);
    } else {
      double g[3];
      if (G3)
        interp_g3<S>(g3, mm, c, g);
      else
        interp_g<S>(phi, mm, c, inv2h, g);
      // finish all three sums here: otherwise the compiler sinks the sums of
      // g[1], g[2] to the kick of their component and keeps every node's
      // loaded force and weight live until then (TSC: 186 registers).  The
      // empty asm only pins the three values to this point.
      asm volatile("" : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]));
      for (int d = 0; d < 3; ++d) {
        PT* p = (PT*)pa.p[d];
        const PT pn = (PT)((double)p_old[d] + g[d] * kick_coef);
        __builtin_nontemporal_store(pn, p + i);
        x[d] = drift_wrap(x[d], (double)pn, drift_coef, mm);
        __builtin_nontemporal_store(x[d], pa.x[d] + i);
      }
      if (count_removed) out = dist2_nofma(x[0], x[1], x[2], o0, o1, o2) > r2;
    }
  }
  if (count_removed) {
    const unsigned long long mask = __ballot(out);
    if ((threadIdx.x & 63) == 0 && mask) atomicAdd(removed_count, (uint32_t)__popcll(mask));
  }
}

// Lightcone crossing of removed particles: the root u in [0, 1] of
// A u^2 + B u + C = 0 with A = w.w - L^2, B = -2 (d.w + r L), C = d.d - r^2
// (d = x1 - x_obs, w = p1 dtau / a1, L = c dtau): |d - u w| = r + u L.  For
// |w| < L (A < 0) and C > 0 there is one positive root, 2 C / (-B + sqrt(D)),
// the cancellation-free form.
// The lightcone record of particle i at out slot j (the crossing root u of
// |x1 - u w - x_obs| = r + u light, w = p1 disp, clamped to [0, 1]).
template <typename PT>
__device__ inline void lc_record(const ParticleArgs& pa, int64_t i, const double o[3], double r,
                                 double light, double disp, double a1, double da,
                                 const LcArgs& out, int64_t j) {
  double d[3], w[3], p[3];
  for (int k = 0; k < 3; ++k) {
    p[k] = (double)((const PT*)pa.p[k])[i];
    d[k] = pa.x[k][i] - o[k];
    w[k] = p[k] * disp;
  }
  const double A = (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) - light * light;
  const double B = -2.0 * ((d[0] * w[0] + d[1] * w[1] + d[2] * w[2]) + r * light);
  const double C = (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - r * r;
  double u = 0.0;
  if (C > 0.0 && light > 0.0) {
    const double den = -B + sqrt(fmax(B * B - 4.0 * A * C, 0.0));
    u = den > 0.0 ? fmin(2.0 * C / den, 1.0) : 1.0;
  }
  out.id[j] = pa.id[i];
  out.a[j] = a1 - u * da;
  for (int k = 0; k < 3; ++k) {
    out.x[k][j] = pa.x[k][i] - u * w[k];
    out.p[k][j] = p[k];
  }
}

template <typename PT>
__global__ void __launch_bounds__(256)
k_lightcone(ParticleArgs pa, int64_t first, int64_t count, double o0, double o1, double o2,
            double r, double light, double disp, double a1, double da, LcArgs out,
            int64_t out_first) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  const double o[3] = {o0, o1, o2};
  lc_record<PT>(pa, first + q, o, r, light, disp, a1, da, out, out_first + q);
}

// Fixed domain: mark[i] = particle i outside the lightcone at the step's
// start (the removal predicate with the previous step's end radius).
__global__ void __launch_bounds__(256)
k_lc_mark(ParticleArgs pa, double o0, double o1, double o2, double r2, uint8_t* __restrict__ mark) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= pa.n) return;
  mark[i] = dist2_nofma(pa.x[0][i], pa.x[1][i], pa.x[2][i], o0, o1, o2) > r2 ? 1 : 0;
}

// Fixed domain: record the particles outside at the step's end that were
// inside at its start, in slots base + (atomic counter), below capacity.
template <typename PT>
__global__ void __launch_bounds__(256)
k_lc_cross(ParticleArgs pa, double o0, double o1, double o2, double r2, double r, double light,
           double disp, double a1, double da, const uint8_t* __restrict__ mark, LcArgs out,
           int64_t base, int64_t capacity, unsigned long long* __restrict__ counter) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= pa.n || mark[i]) return;
  if (!(dist2_nofma(pa.x[0][i], pa.x[1][i], pa.x[2][i], o0, o1, o2) > r2)) return;
  const int64_t j = base + (int64_t)atomicAdd(counter, 1ull);
  if (j >= capacity) return;
  const double o[3] = {o0, o1, o2};
  lc_record<PT>(pa, i, o, r, light, disp, a1, da, out, j);
}

template <int S>
__global__ void __launch_bounds__(256)
k_interp_force(ParticleArgs pa, const double* __restrict__ phi, MeshMap mm, double inv2h,
               double* __restrict__ g0, double* __restrict__ g1, double* __restrict__ g2,
               uint32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= pa.n) return;
  const double x[3] = {pa.x[0][i], pa.x[1][i], pa.x[2][i]};
  Stencil<S> c;
  const uint32_t bad = assign_setup<S>(x, mm, c);
  if (bad) {
    atomicOr(flags, bad);
    return;
  }
  double g[3];
  interp_g<S>(phi, mm, c, inv2h, g);
  g0[i] = g[0];
  g1[i] = g[1];
  g2[i] = g[2];
}

// ------------------------------------------------------------ compaction
// Workgroup b owns particles [b kChunk, (b+1) kChunk) in 4 rounds of 256.
__global__ void __launch_bounds__(256)
k_count_kept(ParticleArgs pa, double o0, double o1, double o2, double r2,
             uint32_t* __restrict__ block_counts) {
  __shared__ uint32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t mine = 0;
  for (int u = 0; u < kChunk / 256; ++u) {
    const int64_t i = base + u * 256 + tid;
    bool keep = false;
    if (i < pa.n) keep = !(dist2_nofma(pa.x[0][i], pa.x[1][i], pa.x[2][i], o0, o1, o2) > r2);
    const unsigned long long mask = __ballot(keep);
    if (lane == 0) mine += (uint32_t)__popcll(mask);
  }
  if (lane == 0) wsum[wave] = mine;
  __syncthreads();
  if (tid == 0) block_counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// The block-start table of the block deposit after a stable compaction: a
// block's first index becomes the number of kept particles before it, the
// kept count of the whole chunks before it plus those kept in its chunk ahead
// of it (the same FP64 predicate as k_count_kept, one wave per block).  Runs
// before the particles move; each wave reads and writes its own entry only.
__global__ void __launch_bounds__(64)
k_block_starts_compact(ParticleArgs pa, double o0, double o1, double o2, double r2,
                       const uint32_t* __restrict__ offsets, const uint64_t* __restrict__ kept_total,
                       int64_t nblk, int64_t* __restrict__ start) {
  const int64_t m = blockIdx.x;
  if (m > nblk) return;
  const int64_t s0 = start[m];
  if (s0 >= pa.n) {
    if (threadIdx.x == 0) start[m] = (int64_t)*kept_total;
    return;
  }
  const int64_t c0 = (s0 / kChunk) * kChunk;
  uint64_t kept = 0;
  for (int64_t i0 = c0; i0 < s0; i0 += 64) {
    const int64_t i = i0 + threadIdx.x;
    const bool keep = i < s0 && !(dist2_nofma(pa.x[0][i], pa.x[1][i], pa.x[2][i], o0, o1, o2) > r2);
    kept += (uint64_t)__popcll(__ballot(keep));
  }
  if (threadIdx.x == 0) start[m] = (int64_t)offsets[s0 / kChunk] + (int64_t)kept;
}

// Exclusive scan of nb block counts by one workgroup; total to *kept_total.
__global__ void __launch_bounds__(1024)
k_scan_counts(const uint32_t* __restrict__ counts, uint32_t* __restrict__ offsets, int64_t nb,
              uint64_t* __restrict__ kept_total) {
  __shared__ uint64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = tid * per, b1 = min(nb, b0 + per);
  uint64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += counts[b];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = tid ? part[tid - 1] : 0;
  for (int64_t b = b0; b < b1; ++b) {
    offsets[b] = (uint32_t)run;
    run += counts[b];
  }
  if (tid == 1023) *kept_total = part[1023];
}

template <typename PT>
__global__ void __launch_bounds__(256)
k_scatter(ParticleArgs pa, double o0, double o1, double o2, double r2,
          const uint32_t* __restrict__ offsets, const uint64_t* __restrict__ kept_total,
          double* __restrict__ sx0, double* __restrict__ sx1, double* __restrict__ sx2,
          PT* __restrict__ sp0, PT* __restrict__ sp1, PT* __restrict__ sp2,
          uint32_t* __restrict__ sid) {
  __shared__ uint32_t wk[4], wr[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  const uint64_t kept_before = offsets[blockIdx.x];
  const uint64_t removed_before = (uint64_t)base - kept_before;
  const uint64_t nkept = *kept_total;
  const unsigned long long below = (1ull << lane) - 1ull;
  uint64_t run_k = 0, run_r = 0;
  for (int u = 0; u < kChunk / 256; ++u) {
    const int64_t i = base + u * 256 + tid;
    const bool valid = i < pa.n;
    bool keep = false;
    if (valid) keep = !(dist2_nofma(pa.x[0][i], pa.x[1][i], pa.x[2][i], o0, o1, o2) > r2);
    const unsigned long long mk = __ballot(keep);
    const unsigned long long mr = __ballot(valid && !keep);
    if (lane == 0) {
      wk[wave] = (uint32_t)__popcll(mk);
      wr[wave] = (uint32_t)__popcll(mr);
    }
    __syncthreads();
    uint32_t ok = 0, orr = 0;
    for (int w = 0; w < wave; ++w) {
      ok += wk[w];
      orr += wr[w];
    }
    const uint32_t tk = wk[0] + wk[1] + wk[2] + wk[3];
    const uint32_t tr = wr[0] + wr[1] + wr[2] + wr[3];
    if (valid) {
      uint64_t dst;
      if (keep)
        dst = kept_before + run_k + ok + (uint64_t)__popcll(mk & below);
      else
        dst = nkept + removed_before + run_r + orr + (uint64_t)__popcll(mr & below);
      sx0[dst] = pa.x[0][i];
      sx1[dst] = pa.x[1][i];
      sx2[dst] = pa.x[2][i];
      sp0[dst] = ((const PT*)pa.p[0])[i];
      sp1[dst] = ((const PT*)pa.p[1])[i];
      sp2[dst] = ((const PT*)pa.p[2])[i];
      sid[dst] = pa.id[i];
    }
    run_k += tk;
    run_r += tr;
    __syncthreads();
  }
}

// Deposit right after a re-sort into blocks of kBlkCells^3 cells: the
// particles of a block are contiguous (block_start, in the blocks' Morton
// order), and one workgroup of 1024 threads takes one block.  Its LDS window
// is fixed in advance: the block, kBlkMargin<S> cells of drift on each side,
// and the reach of the S^3 stencil; a particle whose nodes leave it (one
// that drifted further since the sort) goes to global atomics, so every
// routing gives the same integer sums.  Windows of neighbouring blocks
// overlap only in those margins, and no workgroup needs a bounding box
// (reductions, barriers) or straddles two blocks.
template <int S>
struct BlkWin {
  static constexpr int M = S == 2 ? 2 : 1;                  // drift margin, cells
  static constexpr int W = kBlkCells + 2 * M + 2 * S - 3;   // 21 for both stencils
  static constexpr int L = M + S - 2;                       // window start below the block
};

__device__ inline uint32_t compact3(uint32_t v) {
  // the inverse of spread3 on every third bit
  v &= 0x49249249;
  v = (v | (v >> 2)) & 0x430c30c3;
  v = (v | (v >> 4)) & 0x0700f00f;
  v = (v | (v >> 8)) & 0x070000ff;
  v = (v | (v >> 16)) & 0x7ff;
  return v;
}

template <typename PT, bool DRIFT, int S>
__global__ void __launch_bounds__(1024)
k_block_deposit(ParticleArgs pa, double coef, MeshMap mm, const int64_t* __restrict__ start,
                unsigned long long* __restrict__ counts, uint32_t* __restrict__ flags) {
  constexpr int W = BlkWin<S>::W;
  __shared__ unsigned long long acc[W * W * W];
  const int64_t b = xcd_block();
  const int64_t s0 = start[b], s1 = start[b + 1];
  if (s0 >= s1) return;                        // an empty block (uniform)
  const uint32_t mb = (uint32_t)b;
  const int lo0 = (int)compact3(mb) * kBlkCells - BlkWin<S>::L;
  const int lo1 = (int)compact3(mb >> 1) * kBlkCells - BlkWin<S>::L;
  const int lo2 = (int)compact3(mb >> 2) * kBlkCells - BlkWin<S>::L;
  for (int q = threadIdx.x; q < W * W * W; q += 1024) acc[q] = 0ull;
  __syncthreads();
  const int m = mm.ng - 1, half = mm.ng >> 1;
  uint32_t bad_all = 0;
  for (int64_t i = s0 + threadIdx.x; i < s1; i += 1024) {
    double x[3];
    for (int d = 0; d < 3; ++d) {
      double v = __builtin_nontemporal_load(pa.x[d] + i);
      if (DRIFT) v = drift_wrap(v, (double)__builtin_nontemporal_load((const PT*)pa.p[d] + i), coef, mm);
      x[d] = v;
    }
    Frac c;
    const uint32_t bad = assign_frac<S>(x, mm, c);
    if (bad) {
      bad_all |= bad;
      continue;
    }
    uint64_t wt[3][S];
    for (int d = 0; d < 3; ++d) axis_weights<S>(c.f[d], mm.frac_bits, wt[d]);
    int r0 = c.cell[0] - lo0, r1 = c.cell[1] - lo1, r2 = c.cell[2] - lo2;
    if (mm.periodic) {
      r0 = ((r0 + half) & m) - half;
      r1 = ((r1 + half) & m) - half;
      r2 = ((r2 + half) & m) - half;
    }
    if ((unsigned)r0 <= (unsigned)(W - S) && (unsigned)r1 <= (unsigned)(W - S) &&
        (unsigned)r2 <= (unsigned)(W - S)) {
      for (int dz = 0; dz < S; ++dz)
        for (int dy = 0; dy < S; ++dy) {
          const uint64_t wyz = wt[1][dy] * wt[2][dz];
          if (wyz == 0) continue;
          const int row = ((r2 + dz) * W + r1 + dy) * W + r0;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = wt[0][dx] * wyz;
            if (wgt) atomicAdd(&acc[row + dx], (unsigned long long)wgt);
          }
        }
    } else {
      for (int dz = 0; dz < S; ++dz) {
        int kk = c.cell[2] + dz;
        if (mm.periodic) kk &= m;
        for (int dy = 0; dy < S; ++dy) {
          int jj = c.cell[1] + dy;
          if (mm.periodic) jj &= m;
          const uint64_t wyz = wt[1][dy] * wt[2][dz];
          if (wyz == 0) continue;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = wt[0][dx] * wyz;
            if (wgt == 0) continue;
            int ii = c.cell[0] + dx;
            if (mm.periodic) ii &= m;
            atomicAdd(counts + lin(ii, jj, kk, mm.ng), (unsigned long long)wgt);
          }
        }
      }
    }
  }
  if (bad_all) atomicOr(flags, bad_all);
  __syncthreads();
  for (int q = threadIdx.x; q < W * W * W; q += 1024) {
    const unsigned long long v = acc[q];
    if (!v) continue;
    int gx = lo0 + q % W, gy = lo1 + (q / W) % W, gz = lo2 + q / (W * W);
    if (mm.periodic) {
      gx &= m;
      gy &= m;
      gz &= m;
    }
    atomicAdd(counts + lin(gx, gy, gz, mm.ng), v);
  }
}

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

template <typename PT>
void launch_drift_deposit(const ParticleArgs& pa, double drift_coef, int drift,
                          const MeshMap& mm, uint64_t* counts, uint32_t* flags, hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_DEPOSIT);
  const dim3 g(grid_for(pa.n, kDepThreads * kDepPer));
  unsigned long long* cu = (unsigned long long*)counts;
#define SDPM_DEP(D, S)                                                                         \
  hipLaunchKernelGGL((k_drift_deposit<PT, D, S>), g, dim3(kDepThreads), 0, st, pa, drift_coef, mm, \
                     cu, flags)
  if (mm.tsc) {
    if (drift) SDPM_DEP(true, 3); else SDPM_DEP(false, 3);
  } else {
    if (drift) SDPM_DEP(true, 2); else SDPM_DEP(false, 2);
  }
#undef SDPM_DEP
  // positions (and with the drift the momenta) read; the drifted positions
  // are not written back
  const double per = drift ? 24.0 + 3.0 * sizeof(PT) : 24.0;
  prof_end(st, K_DEPOSIT, per * pa.n + 8.0 * box_cells(mm.active));
}

template <typename PT>
void launch_block_deposit(const ParticleArgs& pa, double drift_coef, int drift, const MeshMap& mm,
                          const int64_t* block_start, uint64_t* counts, uint32_t* flags,
                          hipStream_t st) {
  if (pa.n <= 0) return;
  const int64_t nb1 = mm.ng >> kBlkShift;
  const dim3 g((unsigned)(nb1 * nb1 * nb1));
  unsigned long long* cu = (unsigned long long*)counts;
  prof_begin(st, K_DEPOSIT);
#define SDPM_BDEP(D, S)                                                                         \
  hipLaunchKernelGGL((k_block_deposit<PT, D, S>), g, dim3(1024), 0, st, pa, drift_coef, mm,      \
                     block_start, cu, flags)
  if (mm.tsc) {
    if (drift) SDPM_BDEP(true, 3); else SDPM_BDEP(false, 3);
  } else {
    if (drift) SDPM_BDEP(true, 2); else SDPM_BDEP(false, 2);
  }
#undef SDPM_BDEP
  // the same algorithmic bytes as launch_drift_deposit
  const double per = drift ? 24.0 + 3.0 * sizeof(PT) : 24.0;
  prof_end(st, K_DEPOSIT, per * pa.n + 8.0 * box_cells(mm.active));
}
template void launch_block_deposit<float>(const ParticleArgs&, double, int, const MeshMap&,
                                          const int64_t*, uint64_t*, uint32_t*, hipStream_t);
template void launch_block_deposit<double>(const ParticleArgs&, double, int, const MeshMap&,
                                           const int64_t*, uint64_t*, uint32_t*, hipStream_t);

template void launch_drift_deposit<float>(const ParticleArgs&, double, int, const MeshMap&,
                                          uint64_t*, uint32_t*, hipStream_t);
template void launch_drift_deposit<double>(const ParticleArgs&, double, int, const MeshMap&,
                                           uint64_t*, uint32_t*, hipStream_t);

template <typename PT>
void launch_interp_kick_drift(const ParticleArgs& pa, const double* phi, const float* g3,
                              const MeshMap& mm, double inv2h, double drift0_coef,
                              double kick_coef, double drift_coef, const double* x_obs, double r2,
                              int count_removed, uint32_t* removed_count, uint32_t* flags,
                              hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_INTERP_KICK_DRIFT);
#define SDPM_IKD(G, S)                                                                          \
  hipLaunchKernelGGL((k_interp_kick_drift<PT, G, S>), dim3(grid_for(pa.n, 256)), dim3(256), 0, st, \
                     pa, phi, g3, mm, inv2h, drift0_coef, kick_coef, drift_coef, x_obs[0],        \
                     x_obs[1], x_obs[2],                                                          \
                     r2, count_removed, removed_count, flags)
  if (mm.tsc) {
    if (g3) SDPM_IKD(true, 3); else SDPM_IKD(false, 3);
  } else {
    if (g3) SDPM_IKD(true, 2); else SDPM_IKD(false, 2);
  }
#undef SDPM_IKD
  // particles 36 B read and written; the mesh read once (FP32 force or FP64 potential)
  prof_end(st, K_INTERP_KICK_DRIFT,
           (48.0 + 6.0 * sizeof(PT)) * pa.n + (g3 ? 12.0 : 8.0) * box_cells(mm.active));
}
template void launch_interp_kick_drift<float>(const ParticleArgs&, const double*, const float*,
                                              const MeshMap&, double, double, double, double,
                                              const double*, double, int, uint32_t*, uint32_t*,
                                              hipStream_t);
template void launch_interp_kick_drift<double>(const ParticleArgs&, const double*, const float*,
                                               const MeshMap&, double, double, double, double,
                                               const double*, double, int, uint32_t*, uint32_t*,
                                               hipStream_t);

void launch_interp_force(const ParticleArgs& pa, const double* phi, const MeshMap& mm,
                         double inv2h, double* g0, double* g1, double* g2, uint32_t* flags,
                         hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_INTERP_FORCE);
  if (mm.tsc)
    hipLaunchKernelGGL(k_interp_force<3>, dim3(grid_for(pa.n, 256)), dim3(256), 0, st, pa, phi, mm,
                       inv2h, g0, g1, g2, flags);
  else
    hipLaunchKernelGGL(k_interp_force<2>, dim3(grid_for(pa.n, 256)), dim3(256), 0, st, pa, phi, mm,
                       inv2h, g0, g1, g2, flags);
  prof_end(st, K_INTERP_FORCE, 48.0 * pa.n + 8.0 * box_cells(mm.active));
}

template <typename PT>
void launch_lightcone(const ParticleArgs& pa, int64_t first, int64_t count, const double* x_obs,
                      double r1, double light, double disp, double a1, double da, const LcArgs& out,
                      int64_t out_first, hipStream_t st) {
  if (count <= 0) return;
  prof_begin(st, K_LIGHTCONE);
  hipLaunchKernelGGL(k_lightcone<PT>, dim3(grid_for(count, 256)), dim3(256), 0, st, pa, first, count,
                     x_obs[0], x_obs[1], x_obs[2], r1, light, disp, a1, da, out, out_first);
  // particle read (x, p, id) and record written (id, a, x, p)
  prof_end(st, K_LIGHTCONE, (24.0 + 3.0 * sizeof(PT) + 4.0 + 4.0 + 8.0 + 48.0) * count);
}
template void launch_lightcone<float>(const ParticleArgs&, int64_t, int64_t, const double*, double,
                                      double, double, double, double, const LcArgs&, int64_t,
                                      hipStream_t);
template void launch_lightcone<double>(const ParticleArgs&, int64_t, int64_t, const double*, double,
                                       double, double, double, double, const LcArgs&, int64_t,
                                       hipStream_t);

void launch_lc_mark(const ParticleArgs& pa, const double* x_obs, double r2, uint8_t* mark,
                    hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_LIGHTCONE);
  hipLaunchKernelGGL(k_lc_mark, dim3(grid_for(pa.n, 256)), dim3(256), 0, st, pa, x_obs[0], x_obs[1],
                     x_obs[2], r2, mark);
  prof_end(st, K_LIGHTCONE, 25.0 * pa.n);
}

template <typename PT>
void launch_lc_cross(const ParticleArgs& pa, const double* x_obs, double r2, double r,
                     double light, double disp, double a1, double da, const uint8_t* mark,
                     const LcArgs& out, int64_t base, int64_t capacity,
                     unsigned long long* counter, hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_LIGHTCONE);
  hipLaunchKernelGGL(k_lc_cross<PT>, dim3(grid_for(pa.n, 256)), dim3(256), 0, st, pa, x_obs[0],
                     x_obs[1], x_obs[2], r2, r, light, disp, a1, da, mark, out, base, capacity,
                     counter);
  // positions and marks of all active particles (records: a small fraction)
  prof_end(st, K_LIGHTCONE, 25.0 * pa.n);
}
template void launch_lc_cross<float>(const ParticleArgs&, const double*, double, double, double,
                                     double, double, double, const uint8_t*, const LcArgs&,
                                     int64_t, int64_t, unsigned long long*, hipStream_t);
template void launch_lc_cross<double>(const ParticleArgs&, const double*, double, double, double,
                                      double, double, double, const uint8_t*, const LcArgs&,
                                      int64_t, int64_t, unsigned long long*, hipStream_t);

template <typename PT>
void launch_compact(const ParticleArgs& pa, const double* x_obs, double r2, void* scratch,
                    uint32_t* block_counts, uint32_t* block_offsets, uint64_t* kept_total,
                    int64_t* block_start, int64_t nblk, hipStream_t st) {
  if (pa.n <= 0) return;
  const int64_t nb = (pa.n + kChunk - 1) / kChunk;
  prof_begin(st, K_COUNT_KEPT);
  hipLaunchKernelGGL(k_count_kept, dim3((unsigned)nb), dim3(256), 0, st, pa, x_obs[0], x_obs[1],
                     x_obs[2], r2, block_counts);
  prof_end(st, K_COUNT_KEPT, 24.0 * pa.n);
  prof_begin(st, K_SCAN);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, block_counts, block_offsets, nb,
                     kept_total);
  prof_end(st, K_SCAN, 8.0 * nb);
  if (block_start)
    hipLaunchKernelGGL(k_block_starts_compact, dim3((unsigned)(nblk + 1)), dim3(64), 0, st, pa,
                       x_obs[0], x_obs[1], x_obs[2], r2, block_offsets, kept_total, nblk,
                       block_start);
  char* s = (char*)scratch;
  const size_t n = (size_t)pa.n;
  double* sx0 = (double*)s;
  double* sx1 = sx0 + n;
  double* sx2 = sx1 + n;
  PT* sp0 = (PT*)(sx2 + n);
  PT* sp1 = sp0 + n;
  PT* sp2 = sp1 + n;
  uint32_t* sid = (uint32_t*)(sp2 + n);
  const double pbytes = (24.0 + 3.0 * sizeof(PT) + 4.0) * pa.n;
  prof_begin(st, K_SCATTER);
  hipLaunchKernelGGL(k_scatter<PT>, dim3((unsigned)nb), dim3(256), 0, st, pa, x_obs[0], x_obs[1],
                     x_obs[2], r2, block_offsets, kept_total, sx0, sx1, sx2, sp0, sp1, sp2, sid);
  prof_end(st, K_SCATTER, 2.0 * pbytes);
  prof_begin(st, K_COPY);
  for (int d = 0; d < 3; ++d) {
    (void)hipMemcpyAsync(pa.x[d], sx0 + d * n, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(pa.p[d], sp0 + d * n, n * sizeof(PT), hipMemcpyDeviceToDevice, st);
  }
  (void)hipMemcpyAsync(pa.id, sid, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  prof_end(st, K_COPY, 2.0 * pbytes);
}
template void launch_compact<float>(const ParticleArgs&, const double*, double, void*, uint32_t*,
                                    uint32_t*, uint64_t*, int64_t*, int64_t, hipStream_t);
template void launch_compact<double>(const ParticleArgs&, const double*, double, void*, uint32_t*,
                                     uint32_t*, uint64_t*, int64_t*, int64_t, hipStream_t);

}  // namespace sdpm
