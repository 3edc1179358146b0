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
// periodic mesh, where the users wrap it with & (ng - 1)) and the weights.
template <int S>
struct Stencil {
  int cell[3];
  uint64_t w[3][S];
};

// Fixed-point coordinates and weights of one particle.  Returns 0 or a
// kFlag* bit (then the stencil is a harmless one-node placeholder).
template <int S>
__device__ inline uint32_t assign_setup(const double x[3], const MeshMap& mm, Stencil<S>& c) {
  const int64_t span = (int64_t)mm.ng << mm.frac_bits;
  const uint64_t one = 1ull << mm.frac_bits;
  uint32_t bad = 0;
  for (int d = 0; d < 3; ++d) {
    const double u = x[d] * mm.scale;
    const bool nan_or_inf = u != u || __builtin_isinf(u);
    if (nan_or_inf || !(u >= 0.0 && u <= (double)span)) {
      bad |= nan_or_inf ? kFlagOverflow : kFlagDomain;
      c.cell[d] = 0;
      c.w[d][0] = one;
      for (int t = 1; t < S; ++t) c.w[d][t] = 0;
      continue;
    }
    int64_t U = (int64_t)floor(u);
    if (mm.periodic) U &= span - 1;
    if constexpr (S == 2) {
      c.cell[d] = (int)(U >> mm.frac_bits);
      const uint64_t q = (uint64_t)U & (one - 1);
      c.w[d][0] = one - q;
      c.w[d][1] = q;
    } else {
      const int64_t half = (int64_t)one >> 1;
      const int64_t node = (U + half) >> mm.frac_bits;
      const int64_t D = U - (node << mm.frac_bits);
      const uint64_t wm = (uint64_t)((half - D) * (half - D) + (int64_t)one) >> (mm.frac_bits + 1);
      const uint64_t wp = (uint64_t)((half + D) * (half + D) + (int64_t)one) >> (mm.frac_bits + 1);
      c.cell[d] = (int)node - 1;
      c.w[d][0] = wm;
      c.w[d][1] = one - wm - wp;
      c.w[d][2] = wp;
    }
    if (!mm.periodic && (c.cell[d] < mm.active.lo[d] || c.cell[d] + S - 1 > mm.active.hi[d]))
      bad |= kFlagDomain;
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

// Drift + deposit, 1024 particles per workgroup.  When the CIC cells of the
// workgroup's particles fit a box of at most LDS cells the weights are summed
// with 64-bit LDS atomics and each touched cell is flushed with one global
// atomic; otherwise every corner goes straight to global atomics.  Integer
// sums: the result is the same either way and in any order.  Two tile sizes:
// kDepLds cells (32 KB) fit the particles of a workgroup while they stay near
// their lattice order inside a sort block; once they have moved about a
// whole 16^3-cell block apart its 17^3-cell box needs kDepLdsBig (48 KB,
// fewer workgroups per CU).  Workgroups whose box exceeds kDepLds are counted
// in flags[2] so that the caller can choose the tile for the next deposit.
constexpr int kDepPer = 4;
constexpr int kDepLds = 4096, kDepLdsBig = 6144;

__device__ inline int wave_min(int v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_down(v, off, 64));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_down(v, off, 64));
  return v;
}

template <typename PT, bool DRIFT, int LDS, int S>
__global__ void __launch_bounds__(256)
k_drift_deposit(ParticleArgs pa, double coef, MeshMap mm, unsigned long long* __restrict__ counts,
                uint32_t* __restrict__ flags) {
  __shared__ unsigned long long acc[LDS];
  __shared__ int blo[3], bhi[3];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * (256 * kDepPer);
  if (tid < 3) {
    blo[tid] = 0x7fffffff;
    bhi[tid] = -0x7fffffff;
  }
  Stencil<S> c[kDepPer];
  bool ok[kDepPer];
  int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
  uint32_t bad_all = 0;
#pragma unroll
  for (int u = 0; u < kDepPer; ++u) {
    const int64_t i = base + u * 256 + tid;
    ok[u] = false;
    if (i >= pa.n) continue;
    double x[3];
    for (int d = 0; d < 3; ++d) {
      double v = __builtin_nontemporal_load(pa.x[d] + i);
      if (DRIFT) {
        v = drift_nofma(v, (double)__builtin_nontemporal_load((const PT*)pa.p[d] + i), coef);
        if (mm.periodic) {
          if (v < 0.0) v += mm.box;
          if (v >= mm.box) v -= mm.box;
        }
        __builtin_nontemporal_store(v, pa.x[d] + i);
      }
      x[d] = v;
    }
    const uint32_t bad = assign_setup<S>(x, mm, c[u]);
    if (bad) {
      bad_all |= bad;
      continue;
    }
    ok[u] = true;
    for (int d = 0; d < 3; ++d) {
      mn[d] = min(mn[d], c[u].cell[d]);
      mx[d] = max(mx[d], c[u].cell[d]);
    }
  }
  if (bad_all) atomicOr(flags, bad_all);
  __syncthreads();
  for (int d = 0; d < 3; ++d) {
    const int a = wave_min(mn[d]), b = wave_max(mx[d]);
    if ((tid & 63) == 0) {
      atomicMin(&blo[d], a);
      atomicMax(&bhi[d], b);
    }
  }
  __syncthreads();
  const int lx = bhi[0] - blo[0] + S, ly = bhi[1] - blo[1] + S, lz = bhi[2] - blo[2] + S;
  if (lx < S) return;                                    // no valid particle in the workgroup
  const int m = mm.ng - 1;
  const int64_t vol_box = (int64_t)lx * ly * lz;
  if (tid == 0 && vol_box > kDepLds) atomicAdd(flags + 2, 1u);
  const bool use_lds = vol_box <= LDS;
  if (use_lds) {
    const int vol = lx * ly * lz;
    for (int q = tid; q < vol; q += 256) acc[q] = 0ull;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kDepPer; ++u) {
      if (!ok[u]) continue;
      const int ax = c[u].cell[0] - blo[0], ay = c[u].cell[1] - blo[1], az = c[u].cell[2] - blo[2];
      for (int dz = 0; dz < S; ++dz)
        for (int dy = 0; dy < S; ++dy) {
          const uint64_t wyz = c[u].w[1][dy] * c[u].w[2][dz];
          if (wyz == 0) continue;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = c[u].w[0][dx] * wyz;
            if (wgt) atomicAdd(&acc[((az + dz) * ly + ay + dy) * lx + ax + dx], (unsigned long long)wgt);
          }
        }
    }
    __syncthreads();
    for (int q = tid; q < vol; q += 256) {
      const unsigned long long v = acc[q];
      if (!v) continue;
      int gx = blo[0] + q % lx, gy = blo[1] + (q / lx) % ly, gz = blo[2] + q / (lx * ly);
      if (mm.periodic) {
        gx &= m;
        gy &= m;
        gz &= m;
      }
      atomicAdd(counts + lin(gx, gy, gz, mm.ng), v);
    }
  } else {
#pragma unroll
    for (int u = 0; u < kDepPer; ++u) {
      if (!ok[u]) continue;
      for (int dz = 0; dz < S; ++dz) {
        const int kk = mm.periodic ? ((c[u].cell[2] + dz) & m) : c[u].cell[2] + dz;
        for (int dy = 0; dy < S; ++dy) {
          const int jj = mm.periodic ? ((c[u].cell[1] + dy) & m) : c[u].cell[1] + dy;
          const uint64_t wyz = c[u].w[1][dy] * c[u].w[2][dz];
          if (wyz == 0) continue;
          for (int dx = 0; dx < S; ++dx) {
            const uint64_t wgt = c[u].w[0][dx] * wyz;
            if (wgt == 0) continue;
            const int ii = mm.periodic ? ((c[u].cell[0] + dx) & m) : c[u].cell[0] + dx;
            atomicAdd(counts + lin(ii, jj, kk, mm.ng), (unsigned long long)wgt);
          }
        }
      }
    }
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

template <typename PT, bool G3, int S>
__global__ void __launch_bounds__(256)
k_interp_kick_drift(ParticleArgs pa, const double* __restrict__ phi, const float* __restrict__ g3,
                    MeshMap mm, double inv2h,
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
    Stencil<S> c;
    const uint32_t bad = assign_setup<S>(x, mm, c);
    if (bad) {
      atomicOr(flags, bad);
    } else {
      double g[3];
      if (G3)
        interp_g3<S>(g3, mm, c, g);
      else
        interp_g<S>(phi, mm, c, inv2h, g);
      for (int d = 0; d < 3; ++d) {
        PT* p = (PT*)pa.p[d];
        const PT pn = (PT)((double)p_old[d] + g[d] * kick_coef);
        __builtin_nontemporal_store(pn, p + i);
        double v = drift_nofma(x[d], (double)pn, drift_coef);
        if (mm.periodic) {
          if (v < 0.0) v += mm.box;
          if (v >= mm.box) v -= mm.box;
        }
        __builtin_nontemporal_store(v, pa.x[d] + i);
        x[d] = v;
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

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

template <typename PT>
void launch_drift_deposit(const ParticleArgs& pa, double drift_coef, int drift,
                          const MeshMap& mm, uint64_t* counts, uint32_t* flags, bool big_tile,
                          hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_DEPOSIT);
  const dim3 g(grid_for(pa.n, 256 * kDepPer));
  unsigned long long* cu = (unsigned long long*)counts;
#define SDPM_DEP(D, L, S)                                                                       \
  hipLaunchKernelGGL((k_drift_deposit<PT, D, L, S>), g, dim3(256), 0, st, pa, drift_coef, mm, cu, \
                     flags)
  if (mm.tsc) {
    if (drift) {
      if (big_tile) SDPM_DEP(true, kDepLdsBig, 3); else SDPM_DEP(true, kDepLds, 3);
    } else {
      if (big_tile) SDPM_DEP(false, kDepLdsBig, 3); else SDPM_DEP(false, kDepLds, 3);
    }
  } else if (drift) {
    if (big_tile) SDPM_DEP(true, kDepLdsBig, 2); else SDPM_DEP(true, kDepLds, 2);
  } else {
    if (big_tile) SDPM_DEP(false, kDepLdsBig, 2); else SDPM_DEP(false, kDepLds, 2);
  }
#undef SDPM_DEP
  const double per = drift ? 48.0 + 3.0 * sizeof(PT) : 24.0;
  prof_end(st, K_DEPOSIT, per * pa.n + 8.0 * box_cells(mm.active));
}

int64_t deposit_workgroups(int64_t n) { return (n + 256 * kDepPer - 1) / (256 * kDepPer); }
template void launch_drift_deposit<float>(const ParticleArgs&, double, int, const MeshMap&,
                                          uint64_t*, uint32_t*, bool, hipStream_t);
template void launch_drift_deposit<double>(const ParticleArgs&, double, int, const MeshMap&,
                                           uint64_t*, uint32_t*, bool, hipStream_t);

template <typename PT>
void launch_interp_kick_drift(const ParticleArgs& pa, const double* phi, const float* g3,
                              const MeshMap& mm, double inv2h, double kick_coef, double drift_coef,
                              const double* x_obs, double r2, int count_removed,
                              uint32_t* removed_count, uint32_t* flags, hipStream_t st) {
  if (pa.n <= 0) return;
  prof_begin(st, K_INTERP_KICK_DRIFT);
#define SDPM_IKD(G, S)                                                                          \
  hipLaunchKernelGGL((k_interp_kick_drift<PT, G, S>), dim3(grid_for(pa.n, 256)), dim3(256), 0, st, \
                     pa, phi, g3, mm, inv2h, kick_coef, drift_coef, x_obs[0], x_obs[1], x_obs[2],  \
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
                                              const MeshMap&, double, double, double,
                                              const double*, double, int, uint32_t*, uint32_t*,
                                              hipStream_t);
template void launch_interp_kick_drift<double>(const ParticleArgs&, const double*, const float*,
                                               const MeshMap&, double, double, double,
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
                    hipStream_t st) {
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
                                    uint32_t*, uint64_t*, hipStream_t);
template void launch_compact<double>(const ParticleArgs&, const double*, double, void*, uint32_t*,
                                     uint32_t*, uint64_t*, hipStream_t);

}  // namespace sdpm
