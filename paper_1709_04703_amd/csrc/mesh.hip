// Mesh kernels: source assembly, FP64 residual / correction / reductions and
// the multigrid V-cycle (red-black Gauss-Seidel, full-weighting restriction,
// trilinear prolongation, single-workgroup coarsest solve in LDS).
//
// The operator on level l (spacing 2^l h, in units of the fine h^2) is
//   A_l e = (sum of 6 neighbours - 6 e) / 4^l - kappa h^2 e,
// the mesh form of (Lap - kappa) from the implicit step of the paper's
// diffusion equation (Sec. 2.1 Eq. 4; kappa = 0 gives Eq. 3).  Cells outside
// a level's active box keep e = 0 (homogeneous Dirichlet for corrections);
// periodic levels cover the whole mesh and wrap indices with n - 1 masks
// (n is a power of two).  In Dirichlet mode every box satisfies 1 <= lo and
// hi <= n - 2, so the same masked indexing never wraps there.
#include <algorithm>
#include <cmath>
#include <utility>

#include "internal.h"

namespace sdpm {
namespace {

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Deterministic sum over a workgroup of NT threads (NT multiple of 64):
// fixed shuffle tree per wave, then the wave partials in order.  The result
// is valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  v = wave_sum(v);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int w = 0; w < NT / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Multigrid arrays (e, r, t of every level) are stored split by colour:
// the n^3/2 red cells ((i+j+k) even) first, then the black ones, each in
// row order with x index i >> 1.  A colour sweep then streams contiguous,
// fully used cache lines.
__host__ __device__ inline int64_t half_cells(int n) { return (int64_t)n * n * (n >> 1); }
__host__ __device__ inline int64_t sidx(int i, int j, int k, int n) {
  return (int64_t)((i + j + k) & 1) * half_cells(n) + ((int64_t)k * n + j) * (n >> 1) + (i >> 1);
}

// Aligned vectors of 2 and 4 values (one wide load or store).
template <typename T>
struct alignas(2 * sizeof(T)) Vec2 {
  T v[2];
};

template <typename T>
struct alignas(4 * sizeof(T)) Vec4 {
  T v[4];
};

// Streamed 4-wide loads and stores with the non-temporal hint: for arrays
// read or written once per pass and far larger than L2, so that they do not
// displace the data a pass does re-read (stencil neighbours).
template <typename T>
__device__ inline Vec4<T> ld_stream4(const T* p) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const v4 t = __builtin_nontemporal_load((const v4*)p);
  Vec4<T> r;
  r.v[0] = t.x, r.v[1] = t.y, r.v[2] = t.z, r.v[3] = t.w;
  return r;
}
template <typename T>
__device__ inline T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ inline void st_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }
template <typename T>
__device__ inline void st_stream4(T* p, const Vec4<T>& v) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  v4 t;
  t.x = v.v[0], t.y = v.v[1], t.z = v.v[2], t.w = v.v[3];
  __builtin_nontemporal_store(t, (v4*)p);
}

__device__ inline int block_linear() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// x neighbours across lanes.  The vector kernels give each lane 4
// consecutive entries of a row and lay a row segment over the W = blockDim.x
// lanes of one wave (W <= 64), so the entry just before a lane's vector is
// the last entry of the lane before it and the entry just after is the
// first of the lane after it.  Taking them from those lanes' registers
// spares two narrow loads per lane and row that touch the same cache lines
// as the vector loads (FP64 residual at 512^3: 679 -> 541 us).  Lanes at a
// segment's ends, or whose neighbour lane lies outside the box, still load.
template <int W, typename T>
__device__ inline T lane_prev(T v) { return __shfl_up(v, 1u, W); }
template <int W, typename T>
__device__ inline T lane_next(T v) { return __shfl_down(v, 1u, W); }

// Workgroup -> tile mapping.  Box kernels launch a 1-D grid of gx*gy*gz
// workgroups.  The hardware hands consecutive workgroup ids to the 8 XCDs in
// turn; the ids are remapped so that each XCD receives one contiguous run of
// tiles (x fastest, then y, then z), and neighbouring tiles - which read each
// other's halo planes - share that XCD's L2.
struct Tile {
  int bx, by, bz;
};
__device__ inline Tile tile_of(int gx, int gy) {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  const int l = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  Tile t;
  t.bx = l % gx;
  const int q = l / gx;
  t.by = q % gy;
  t.bz = q / gy;
  return t;
}
// tiles of kBoxTx cells (or half-row entries) in x, kBoxTy rows, kBoxKz planes
__device__ inline Tile tile_box(const Box& b) {
  return tile_of((b.hi[0] - b.lo[0] + kBoxTx) / kBoxTx, (b.hi[1] - b.lo[1] + kBoxTy) / kBoxTy);
}
__device__ inline Tile tile_half(const Box& b) {
  return tile_of(((b.hi[0] >> 1) - (b.lo[0] >> 1) + kBoxTx) / kBoxTx,
                 (b.hi[1] - b.lo[1] + kBoxTy) / kBoxTy);
}

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ a, int n, Box b, T v) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) a[lin(i, j, k, n)] = v;
}

// ----------------------------------------------------------- FP64 kernels
// rhs = C * c_scale - c_off - kappa phi ; partial sum of rhs^2.
template <bool CHG>
__global__ void __launch_bounds__(256)
k_rhs(const uint64_t* __restrict__ counts, double* __restrict__ phi, double* __restrict__ rhs,
      int n, Box b, double c_scale, double c_off, double kappa, float* __restrict__ chg,
      double chg_scale, int apply, double* __restrict__ partial) {
  __shared__ double sh[4];
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    for (int k = k0; k <= k1; ++k) {
      const int64_t c = lin(i, j, k, n);
      const double old = phi[c];
      const double v = (double)ld_stream(counts + c) * c_scale - c_off - kappa * old;
      st_stream(rhs + c, v);
      acc += v * v;
      if (CHG) {
        // extrapolated start: phi += the scaled change of the previous solve,
        // which also starts this solve's running change
        const float dv = apply ? (float)(chg_scale * (double)ld_stream(chg + c)) : 0.f;
        if (apply) phi[c] = old + (double)dv;
        st_stream(chg + c, dv);
      }
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// r = rhs - (Lap_h phi - kappa phi) in FP64, stored as T (colour-split).
// Each thread walks kBoxKz planes and carries phi at k-1 and k in registers.
// Partial sum of r^2 per workgroup.
template <typename T>
__global__ void __launch_bounds__(256)
k_residual(const double* __restrict__ phi, const double* __restrict__ rhs, T* __restrict__ rout,
           int n, Box b, double kappa, double* __restrict__ partial) {
  __shared__ double sh[4];
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  const int m = n - 1;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    const int ip = (i + 1) & m, im = (i - 1) & m, jp = (j + 1) & m, jm = (j - 1) & m;
    double below = phi[lin(i, j, (k0 - 1) & m, n)], ctr = phi[lin(i, j, k0, n)];
    for (int k = k0; k <= k1; ++k) {
      const double above = phi[lin(i, j, (k + 1) & m, n)];
      const int64_t c = lin(i, j, k, n);
      const double nb = phi[lin(ip, j, k, n)] + phi[lin(im, j, k, n)] + phi[lin(i, jp, k, n)] +
                        phi[lin(i, jm, k, n)] + above + below;
      const double res = rhs[c] - (nb - 6.0 * ctr - kappa * ctr);
      rout[sidx(i, j, k, n)] = (T)res;
      acc += res * res;
      below = ctr;
      ctr = above;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// k_residual with 4 consecutive cells per thread (vector loads of phi and
// rhs, two 2-wide stores per colour of r).  Vectors start at multiples of 4
// (the box's first x index rounded down); cells outside the box are masked.
// A tile is 4 TXV cells x 256 / TXV rows x kResKz planes.
#ifndef SDPM_RES_KZ
#define SDPM_RES_KZ 16
#endif
// planes per thread of the FP64 residual's z-march (at 512^3, 16 measured 2 %
// faster than 8 and 5 % faster than 4); its 256-thread tiles then span at
// least as many cells as the box kernels', whose grid sizes the reduction
// partials
constexpr int kResKz = SDPM_RES_KZ;
static_assert(kResKz >= 2, "more residual workgroups than reduction partials");

template <typename T, int TXV>
__global__ void __launch_bounds__(256)
k_residual_v4(const double* __restrict__ phi, const double* __restrict__ rhs, T* __restrict__ rout,
              int n, Box b, double kappa, double* __restrict__ partial) {
  __shared__ double sh[4];
  constexpr int TY = 256 / TXV;
  const int ib = b.lo[0] & ~3;
  const Tile tl = tile_of((b.hi[0] - ib + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int i0 = ib + (tl.bx * TXV + threadIdx.x) * 4;
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  const int m = n - 1;
  double acc = 0.0;
  if (i0 <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kResKz;
    const int k1 = min(k0 + kResKz - 1, b.hi[2]);
    const int jp = (j + 1) & m, jm = (j - 1) & m, il = (i0 - 1) & m, ir = (i0 + 4) & m;
    const bool full = i0 >= b.lo[0] && i0 + 3 <= b.hi[0];
    const bool lane_l = threadIdx.x > 0, lane_r = threadIdx.x + 1 < TXV && i0 + 4 <= b.hi[0];
    const int hn = n >> 1;
    const int64_t hc = half_cells(n);
    Vec4<double> below = *(const Vec4<double>*)(phi + lin(i0, j, (k0 - 1) & m, n));
    Vec4<double> ctr = *(const Vec4<double>*)(phi + lin(i0, j, k0, n));
    for (int k = k0; k <= k1; ++k) {
      const Vec4<double> above = *(const Vec4<double>*)(phi + lin(i0, j, (k + 1) & m, n));
      const Vec4<double> ym = *(const Vec4<double>*)(phi + lin(i0, jm, k, n));
      const Vec4<double> yp = *(const Vec4<double>*)(phi + lin(i0, jp, k, n));
      // (the hint measured slower here: the rhs rows are read while the
      // neighbouring phi rows are still being reused)
      const Vec4<double> rv = *(const Vec4<double>*)(rhs + lin(i0, j, k, n));
      double xl = lane_prev<TXV>(ctr.v[3]), xr = lane_next<TXV>(ctr.v[0]);
      if (!lane_l) xl = phi[lin(il, j, k, n)];
      if (!lane_r) xr = phi[lin(ir, j, k, n)];
      double res[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double left = q == 0 ? xl : ctr.v[q - 1];
        const double right = q == 3 ? xr : ctr.v[q + 1];
        const double nb = left + right + ym.v[q] + yp.v[q] + above.v[q] + below.v[q];
        res[q] = rv.v[q] - (nb - 6.0 * ctr.v[q] - kappa * ctr.v[q]);
      }
      // cells i0, i0 + 2 have colour (i0 + j + k) & 1, cells i0 + 1, i0 + 3 the
      // other; both pairs sit at half indices i0 / 2, i0 / 2 + 1 of their colour
      const int c0 = (i0 + j + k) & 1;
      const int64_t row = ((int64_t)k * n + j) * hn + (i0 >> 1);
      if (full) {
        Vec2<T> a, bb;
        a.v[0] = (T)res[0];
        a.v[1] = (T)res[2];
        bb.v[0] = (T)res[1];
        bb.v[1] = (T)res[3];
        {
          typedef T v2 __attribute__((ext_vector_type(2)));
          v2 ta, tb;
          ta.x = a.v[0], ta.y = a.v[1], tb.x = bb.v[0], tb.y = bb.v[1];
          __builtin_nontemporal_store(ta, (v2*)(rout + (int64_t)c0 * hc + row));
          __builtin_nontemporal_store(tb, (v2*)(rout + (int64_t)(c0 ^ 1) * hc + row));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += res[q] * res[q];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + q;
          if (i < b.lo[0] || i > b.hi[0]) continue;
          rout[(int64_t)((c0 + q) & 1) * hc + row + (q >> 1)] = (T)res[q];
          acc += res[q] * res[q];
        }
      }
      below = ctr;
      ctr = above;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// Source assembly fused with the first FP64 residual of a multigrid solve,
// on the tiles of k_residual_v4:
//   rhs = c_scale C - c_off - kappa phi_old                (the rhs pass)
//   r   = rhs - (Lap_h phi0 - kappa phi0),  phi0 = phi_old + d,
// d = (float)(chg_scale chg) the extrapolated start from the previous
// solve's change in chg (MODE 2; MODE 1: d = 0 and the running change chg
// cleared; MODE 0: no running change), evaluated on the fly for each cell
// and its six neighbours.  With a start, neither phi nor chg is written here
// (a neighbour's thread may still read them): the solve's first correction,
// or k_apply_start, adds d to phi and makes it the start of the running
// change.  partial[block] = sum of rhs^2,
// partial[nblocks + block] = sum of r^2.  One pass instead of the rhs pass
// and the residual pass: phi and rhs are not read a second time (and with
// the start, phi is not written here).
// FORCE: the pass also writes the FP32 force mesh of phi (the raw values,
// before any start), with the arithmetic and the store pattern of
// k_force_mesh_v4; the second half sub-step's source pass reads the same
// potential the force is taken from, so one pass serves both.
template <typename T, int TXV, int MODE, bool FORCE>
__global__ void __launch_bounds__(256)
k_rhs_residual_v4(const uint64_t* __restrict__ counts, const double* __restrict__ phi,
                  double* __restrict__ rhs, T* __restrict__ rout, float* __restrict__ chg, int n,
                  Box b, double c_scale, double c_off, double kappa, double chg_scale,
                  int nblocks, double* __restrict__ partial, float* __restrict__ g3,
                  double inv2h) {
  __shared__ double sh[4];
  __shared__ __attribute__((aligned(16))) float stage[FORCE ? 12 * 256 : 4];
  constexpr int TY = 256 / TXV;
  const int ib = b.lo[0] & ~3;
  const Tile tl = tile_of((b.hi[0] - ib + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int i0 = ib + (tl.bx * TXV + threadIdx.x) * 4;
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  const int m = n - 1;
  double acc_r = 0.0, acc_b = 0.0;
  // phi0 at four cells from phi_old there (and d, when MODE 2)
  auto start4 = [&](int64_t c, Vec4<double>& raw, Vec4<float>& d) {
    raw = *(const Vec4<double>*)(phi + c);
    if (MODE == 2) {
      const Vec4<float> prev = *(const Vec4<float>*)(chg + c);
#pragma unroll
      for (int q = 0; q < 4; ++q) d.v[q] = (float)(chg_scale * (double)prev.v[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) d.v[q] = 0.f;
    }
  };
  auto start1 = [&](int64_t c) -> double {
    const double v = phi[c];
    return MODE == 2 ? v + (double)(float)(chg_scale * (double)chg[c]) : v;
  };
  if (i0 <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kResKz;
    const int k1 = min(k0 + kResKz - 1, b.hi[2]);
    const int jp = (j + 1) & m, jm = (j - 1) & m, il = (i0 - 1) & m, ir = (i0 + 4) & m;
    const bool full = i0 >= b.lo[0] && i0 + 3 <= b.hi[0];
    const bool lane_l = threadIdx.x > 0, lane_r = threadIdx.x + 1 < TXV && i0 + 4 <= b.hi[0];
    const int hn = n >> 1;
    const int64_t hc = half_cells(n);
    const int seg0 = ib + tl.bx * TXV * 4;          // first cell of this row segment
    const bool row_full = seg0 >= b.lo[0] && seg0 + 4 * TXV - 1 <= b.hi[0];
    Vec4<double> raw, below, ctr, ctr_raw, below_raw;
    Vec4<float> d, ctr_d;
    start4(lin(i0, j, (k0 - 1) & m, n), raw, d);
    if (FORCE) below_raw = raw;
#pragma unroll
    for (int q = 0; q < 4; ++q) below.v[q] = raw.v[q] + (double)d.v[q];
    start4(lin(i0, j, k0, n), ctr_raw, ctr_d);
#pragma unroll
    for (int q = 0; q < 4; ++q) ctr.v[q] = ctr_raw.v[q] + (double)ctr_d.v[q];
    for (int k = k0; k <= k1; ++k) {
      Vec4<double> above_raw, ym, yp, above;
      Vec4<float> above_d;
      start4(lin(i0, j, (k + 1) & m, n), above_raw, above_d);
#pragma unroll
      for (int q = 0; q < 4; ++q) above.v[q] = above_raw.v[q] + (double)above_d.v[q];
      Vec4<double> ym_raw, yp_raw;
      start4(lin(i0, jm, k, n), raw, d);
      if (FORCE) ym_raw = raw;
#pragma unroll
      for (int q = 0; q < 4; ++q) ym.v[q] = raw.v[q] + (double)d.v[q];
      start4(lin(i0, jp, k, n), raw, d);
      if (FORCE) yp_raw = raw;
#pragma unroll
      for (int q = 0; q < 4; ++q) yp.v[q] = raw.v[q] + (double)d.v[q];
      double xl = lane_prev<TXV>(ctr.v[3]), xr = lane_next<TXV>(ctr.v[0]);
      if (!lane_l) xl = start1(lin(il, j, k, n));
      if (!lane_r) xr = start1(lin(ir, j, k, n));
      const int64_t c = lin(i0, j, k, n);
      Vec4<uint64_t> cnt;
      {
        const Vec2<uint64_t> lo2 = *(const Vec2<uint64_t>*)(counts + c);
        const Vec2<uint64_t> hi2 = *(const Vec2<uint64_t>*)(counts + c + 2);
        cnt.v[0] = lo2.v[0], cnt.v[1] = lo2.v[1], cnt.v[2] = hi2.v[0], cnt.v[3] = hi2.v[1];
      }
      double rv[4], res[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rv[q] = (double)cnt.v[q] * c_scale - c_off - kappa * ctr_raw.v[q];
        const double left = q == 0 ? xl : ctr.v[q - 1];
        const double right = q == 3 ? xr : ctr.v[q + 1];
        const double nb = left + right + ym.v[q] + yp.v[q] + above.v[q] + below.v[q];
        res[q] = rv[q] - (nb - 6.0 * ctr.v[q] - kappa * ctr.v[q]);
      }
      const int c0 = (i0 + j + k) & 1;
      const int64_t row = ((int64_t)k * n + j) * hn + (i0 >> 1);
      if (full) {
        Vec4<double> rr;
#pragma unroll
        for (int q = 0; q < 4; ++q) rr.v[q] = rv[q];
        st_stream4(rhs + c, rr);
        if (MODE == 1) st_stream4(chg + c, ctr_d);
        typedef T v2 __attribute__((ext_vector_type(2)));
        v2 ta, tb;
        ta.x = (T)res[0], ta.y = (T)res[2], tb.x = (T)res[1], tb.y = (T)res[3];
        __builtin_nontemporal_store(ta, (v2*)(rout + (int64_t)c0 * hc + row));
        __builtin_nontemporal_store(tb, (v2*)(rout + (int64_t)(c0 ^ 1) * hc + row));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc_r += res[q] * res[q];
          acc_b += rv[q] * rv[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + q;
          if (i < b.lo[0] || i > b.hi[0]) continue;
          rhs[c + q] = rv[q];
          if (MODE == 1) chg[c + q] = 0.f;
          rout[(int64_t)((c0 + q) & 1) * hc + row + (q >> 1)] = (T)res[q];
          acc_r += res[q] * res[q];
          acc_b += rv[q] * rv[q];
        }
      }
      if constexpr (FORCE) {
        double fl = lane_prev<TXV>(ctr_raw.v[3]), fr = lane_next<TXV>(ctr_raw.v[0]);
        if (!lane_l) fl = phi[lin(il, j, k, n)];
        if (!lane_r) fr = phi[lin(ir, j, k, n)];
        float out[12];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double left = q == 0 ? fl : ctr_raw.v[q - 1];
          const double right = q == 3 ? fr : ctr_raw.v[q + 1];
          out[3 * q + 0] = (float)(-(right - left) * inv2h);
          out[3 * q + 1] = (float)(-(yp_raw.v[q] - ym_raw.v[q]) * inv2h);
          out[3 * q + 2] = (float)(-(above_raw.v[q] - below_raw.v[q]) * inv2h);
        }
        float* dst = g3 + 3 * c;
        if (row_full) {
          // as k_force_mesh_v4: the row segment's 48 TXV contiguous bytes
          // staged in LDS and stored as 3 coalesced 16-byte stores per lane
          float* seg = stage + threadIdx.y * (12 * TXV);
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            Vec4<float> o;
            o.v[0] = out[4 * v], o.v[1] = out[4 * v + 1], o.v[2] = out[4 * v + 2], o.v[3] = out[4 * v + 3];
            *(Vec4<float>*)(seg + 12 * threadIdx.x + 4 * v) = o;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          float* gseg = g3 + 3 * lin(i0 - 4 * (int)threadIdx.x, j, k, n);
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            const Vec4<float> o = *(const Vec4<float>*)(seg + 4 * (TXV * v + threadIdx.x));
            st_stream4(gseg + 4 * (TXV * v + threadIdx.x), o);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else if (full) {
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            Vec4<float> o;
            o.v[0] = out[4 * v], o.v[1] = out[4 * v + 1], o.v[2] = out[4 * v + 2], o.v[3] = out[4 * v + 3];
            st_stream4(dst + 4 * v, o);
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (i0 + q >= b.lo[0] && i0 + q <= b.hi[0])
              for (int dd = 0; dd < 3; ++dd) dst[3 * q + dd] = out[3 * q + dd];
        }
        below_raw = ctr_raw;
      }
      below = ctr;
      ctr = above;
      ctr_raw = above_raw;
      ctr_d = above_d;
    }
  }
  const double sb = block_sum<256>(acc_b, sh);
  const double sr = block_sum<256>(acc_r, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    partial[block_linear()] = sb;
    partial[nblocks + block_linear()] = sr;
  }
}

// A pending extrapolated start: d = (float)(chg_scale chg), phi += d, and d
// becomes the running change.
__global__ void __launch_bounds__(256)
k_apply_start(double* __restrict__ phi, float* __restrict__ chg, int n, Box b, double chg_scale) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    const float d = (float)(chg_scale * (double)ld_stream(chg + c));
    phi[c] += (double)d;
    st_stream(chg + c, d);
  }
}

// phi += e; with CHG the same increment is added to the running change.
// PENDING: the extrapolated start d = (float)(chg_scale chg) of the fused
// rhs pass (k_rhs_residual_v4) is not yet in phi nor in chg (which still
// holds the previous solve's change): phi = (phi + d) + e, chg = d + e, the
// roundings of adding d in a separate pass and then e.
template <typename T, bool CHG, bool PENDING>
__global__ void __launch_bounds__(256)
k_correct(double* __restrict__ phi, const T* __restrict__ e, float* __restrict__ chg, int n, Box b,
          double chg_scale) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    const T ev = ld_stream(e + sidx(i, j, k, n));
    if (CHG) {
      float cv = ld_stream(chg + c);
      if (PENDING) {
        cv = (float)(chg_scale * (double)cv);
        phi[c] = (phi[c] + (double)cv) + (double)ev;
      } else {
        phi[c] += (double)ev;
      }
      st_stream(chg + c, cv + (float)ev);
    } else {
      phi[c] += (double)ev;
    }
  }
}

// k_correct with the next residual estimated in the same pass instead of
// an FP64 residual pass: the V-cycles solved A e = r_old for the stored
// residual r_old (type T), so after phi += e the residual of the defect
// equation is r_old - A e up to the rounding of r_old to T and FP64
// rounding, A e evaluated here in FP64 from the stored correction (zero
// outside a Dirichlet box; periodic axes, those the box spans, wrap).  Per
// workgroup the partial sums of the squares of the estimate, of r_old, of
// the new phi and of e (slots 0..3), from which the host bounds the
// distance between the estimate and the FP64 residual.  Tiles as in
// k_residual_v4: 4 consecutive cells per lane (i0 a multiple of 4), a row
// segment over the TXV lanes of a wave, kResKz planes walked with e of
// planes k - 1, k, k + 1 in registers; e and r_old of the lane's cells are
// two 2-wide loads per colour-split row (cells i0, i0 + 2 and i0 + 1,
// i0 + 3), its x neighbours the adjacent lanes' end cells.
template <typename T, int TXV, bool CHG, bool PENDING>
__global__ void __launch_bounds__(256)
k_correct_est_v4(double* __restrict__ phi, const T* __restrict__ e, const T* __restrict__ rold,
                 float* __restrict__ chg, int n, Box b, double chg_scale, double kappa,
                 double* __restrict__ partial) {
  __shared__ double sh[4];
  constexpr int TY = 256 / TXV;
  const int ib = b.lo[0] & ~3;
  const Tile tl = tile_of((b.hi[0] - ib + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int i0 = ib + (tl.bx * TXV + threadIdx.x) * 4;
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  const int m = n - 1, hn = n >> 1;
  const int64_t hc = half_cells(n);
  const bool in = i0 <= b.hi[0] && j <= b.hi[1];
  const bool px = b.lo[0] == 0 && b.hi[0] == m, py = b.lo[1] == 0 && b.hi[1] == m,
             pz = b.lo[2] == 0 && b.hi[2] == m;
  bool cin[4];                                   // the lane's cells inside the box in x
#pragma unroll
  for (int q = 0; q < 4; ++q) cin[q] = i0 + q >= b.lo[0] && i0 + q <= b.hi[0];
  const bool full = cin[0] && cin[3];
  // the neighbour lane holds cell i0 - 1 (i0 + 4) inside the box without wrapping
  const bool sh_l = threadIdx.x > 0, sh_r = threadIdx.x + 1 < TXV && i0 + 4 <= b.hi[0];
  const bool has_l = px || i0 - 1 >= b.lo[0], has_r = px || i0 + 4 <= b.hi[0];
  const bool has_d = py || j > b.lo[1], has_u = py || j < b.hi[1];
  const int il = (i0 - 1) & m, ir = (i0 + 4) & m, jm = (j - 1) & m, jp = (j + 1) & m;
  // colour-split values of cells i0 .. i0 + 3 of row (jj, kk), natural order
  auto ld4 = [&](const T* a, int jj, int kk) {
    const int c0 = (i0 + jj + kk) & 1;
    const int64_t row = ((int64_t)kk * n + jj) * hn + (i0 >> 1);
    const Vec2<T> u = *(const Vec2<T>*)(a + c0 * hc + row);
    const Vec2<T> v = *(const Vec2<T>*)(a + (c0 ^ 1) * hc + row);
    Vec4<T> r;
    r.v[0] = cin[0] ? u.v[0] : (T)0;
    r.v[1] = cin[1] ? v.v[0] : (T)0;
    r.v[2] = cin[2] ? u.v[1] : (T)0;
    r.v[3] = cin[3] ? v.v[1] : (T)0;
    return r;
  };
  auto zero4 = []() {
    Vec4<T> r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r.v[q] = (T)0;
    return r;
  };
  const int k0 = b.lo[2] + tl.bz * kResKz;
  const int k1 = min(k0 + kResKz - 1, b.hi[2]);
  double s_est = 0.0, s_old = 0.0, s_phi = 0.0, s_e = 0.0;
  Vec4<T> below = zero4(), ctr = zero4();
  if (in) {
    if (pz || k0 > b.lo[2]) below = ld4(e, j, (k0 - 1) & m);
    ctr = ld4(e, j, k0);
  }
  for (int k = k0; k <= k1; ++k) {
    const T from_l = lane_prev<TXV>(ctr.v[3]), from_r = lane_next<TXV>(ctr.v[0]);
    Vec4<T> above = zero4();
    if (in) {
      if (pz || k < b.hi[2]) above = ld4(e, j, (k + 1) & m);
      const Vec4<T> ym = has_d ? ld4(e, jm, k) : zero4();
      const Vec4<T> yp = has_u ? ld4(e, jp, k) : zero4();
      const Vec4<T> rv = ld4(rold, j, k);
      T xl = from_l, xr = from_r;
      if (!sh_l) xl = has_l ? e[sidx(il, j, k, n)] : (T)0;
      if (!sh_r) xr = has_r ? e[sidx(ir, j, k, n)] : (T)0;
      const int64_t c = lin(i0, j, k, n);
      double pn[4];
      float cnew[4];
      Vec4<double> ph;
      Vec4<float> cv;
      if (full) {
        ph = *(const Vec4<double>*)(phi + c);
        if (CHG) cv = ld_stream4(chg + c);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ph.v[q] = cin[q] ? phi[c + q] : 0.0;
          if (CHG) cv.v[q] = cin[q] ? chg[c + q] : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T ev = ctr.v[q];
        if (CHG) {
          float d = cv.v[q];
          if (PENDING) {
            d = (float)(chg_scale * (double)d);
            pn[q] = (ph.v[q] + (double)d) + (double)ev;
          } else {
            pn[q] = ph.v[q] + (double)ev;
          }
          cnew[q] = d + (float)ev;
        } else {
          pn[q] = ph.v[q] + (double)ev;
        }
        const double left = q == 0 ? (double)xl : (double)ctr.v[q - 1];
        const double right = q == 3 ? (double)xr : (double)ctr.v[q + 1];
        const double nb = left + right + (double)ym.v[q] + (double)yp.v[q] + (double)above.v[q] +
                          (double)below.v[q];
        const double ec = (double)ev;
        const double est = (double)rv.v[q] - (nb - 6.0 * ec - kappa * ec);
        if (cin[q]) {
          s_est += est * est;
          s_old += (double)rv.v[q] * (double)rv.v[q];
          s_phi += pn[q] * pn[q];
          s_e += ec * ec;
        }
      }
      if (full) {
        Vec4<double> o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o.v[q] = pn[q];
        *(Vec4<double>*)(phi + c) = o;
        if (CHG) {
          Vec4<float> co;
#pragma unroll
          for (int q = 0; q < 4; ++q) co.v[q] = cnew[q];
          st_stream4(chg + c, co);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!cin[q]) continue;
          phi[c + q] = pn[q];
          if (CHG) chg[c + q] = cnew[q];
        }
      }
    }
    below = ctr;
    ctr = above;
  }
  const double a0 = block_sum<256>(s_est, sh);
  const double a1 = block_sum<256>(s_old, sh);
  const double a2 = block_sum<256>(s_phi, sh);
  const double a3 = block_sum<256>(s_e, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const int64_t nb = gridDim.x, w = block_linear();
    partial[w] = a0;
    partial[nb + w] = a1;
    partial[2 * nb + w] = a2;
    partial[3 * nb + w] = a3;
  }
}

__global__ void __launch_bounds__(256)
k_sum_phi(const double* __restrict__ phi, int n, Box b, double* __restrict__ partial) {
  __shared__ double sh[4];
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    for (int k = k0; k <= k1; ++k) acc += phi[lin(i, j, k, n)];
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// phi += v (and chg += v when given).
__global__ void __launch_bounds__(256)
k_add_const(double* __restrict__ phi, float* __restrict__ chg, int n, Box b, double v) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    phi[c] += v;
    if (chg) chg[c] += (float)v;
  }
}

// out[s] = sum of partial[s * nblocks + 0 .. nblocks), fixed order.
__global__ void __launch_bounds__(1024)
k_reduce_final(const double* __restrict__ partial, int nblocks, int nslots,
               double* __restrict__ out) {
  __shared__ double sh[16];
  for (int s = 0; s < nslots; ++s) {
    const double* p = partial + (int64_t)s * nblocks;
    // the first 8 values of the thread loaded together, then added in the
    // same order as the loop after them (the sum does not depend on how
    // the loads are issued)
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = threadIdx.x + 1024 * u;
      v[u] = t < nblocks ? p[t] : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
    for (int t = threadIdx.x + 8 * 1024; t < nblocks; t += 1024) acc += p[t];
    const double r = block_sum<1024>(acc, sh);
    if (threadIdx.x == 0) out[s] = r;
  }
}

// -------------------------------------------------------- multigrid (T)
// One colour of red-black Gauss-Seidel on the split layout.  Threads map to
// (h, j, k) with h the half-row index; the cell of `color` in that pair is
// i = 2h + ((color + j + k) & 1).  Its six neighbours have the other colour:
// x-neighbours at half-row indices ((i -+ 1) & m) >> 1, y/z neighbours at h.
// FIRST: zero initial guess (neighbours are zero; red only).
template <typename T, bool FIRST>
__global__ void __launch_bounds__(256)
k_smooth_color(T* __restrict__ e, const T* __restrict__ r, int n, Box b, int color, T scale,
               T inv_diag) {
  const Tile tl = tile_half(b);
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (j > b.hi[1]) return;
  const int h = (b.lo[0] >> 1) + tl.bx * kBoxTx + threadIdx.x;
  const int m = n - 1, hn = n >> 1;
  const int64_t hc = half_cells(n);
  const int64_t own = (int64_t)color * hc, oth = (int64_t)(color ^ 1) * hc;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m;
  for (int k = k0; k <= k1; ++k) {
    const int i = 2 * h + ((color + j + k) & 1);
    if (i < b.lo[0] || i > b.hi[0]) continue;
    const int64_t row = ((int64_t)k * n + j) * hn;
    const int64_t c = own + row + h;
    if (FIRST) {
      e[c] = -scale * r[c] * inv_diag;
    } else {
      const int kp = (k + 1) & m, km = (k - 1) & m;
      const T nb = e[oth + row + (((i - 1) & m) >> 1)] + e[oth + row + (((i + 1) & m) >> 1)] +
                   e[oth + ((int64_t)k * n + jm) * hn + h] + e[oth + ((int64_t)k * n + jp) * hn + h] +
                   e[oth + ((int64_t)km * n + j) * hn + h] + e[oth + ((int64_t)kp * n + j) * hn + h];
      e[c] = (nb - scale * r[c]) * inv_diag;
    }
  }
}

// The same sweep with 4 consecutive cells of the colour per thread (16-byte
// loads and stores in FP32): the row of the other colour is one vector load
// plus one scalar for the cell beyond the vector's edge, the y / z
// neighbours and r one vector load each.  Vectors start at multiples of 4
// (the box's first half-row index rounded down; n / 2 is a multiple of 4, so
// a vector never leaves its row) and cells outside the box are masked.
// Tiles are 4 TXV half-row entries x 256 / TXV rows x kVecKz planes (one plane
// per thread measured fastest on the 512^3 mesh: more planes cut the grid
// below what hides the HBM latency).
#ifndef SDPM_VEC_KZ
#define SDPM_VEC_KZ 1
#endif
constexpr int kVecKz = SDPM_VEC_KZ;           // planes per thread of the vector colour kernels

template <typename T, bool FIRST, int TXV>
__global__ void __launch_bounds__(256)
k_smooth_color_v4(T* __restrict__ eo, const T* __restrict__ ex, const T* __restrict__ ro, int n,
                  Box b, int color, T scale, T inv_diag) {
  // eo / ro: this colour's half of e / r; ex: the other colour's half of e
  constexpr int TY = 256 / TXV;
  const int hb = (b.lo[0] >> 1) & ~3, hhi = b.hi[0] >> 1;
  const Tile tl = tile_of((hhi - hb + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  const int h0 = hb + (tl.bx * TXV + threadIdx.x) * 4;
  if (j > b.hi[1] || h0 > hhi) return;
  const int m = n - 1, hn = n >> 1;
  const int k0 = b.lo[2] + tl.bz * kVecKz;
  const int k1 = min(k0 + kVecKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m;
#pragma unroll 2
  for (int k = k0; k <= k1; ++k) {
    const int p = (color + j + k) & 1;          // cell q of the vector: i = 2 (h0 + q) + p
    const int64_t row = ((int64_t)k * n + j) * hn;
    // this colour's r and e are streamed once per sweep; the other colour's e
    // is what the neighbours re-read, so only it is left to the caches
    const Vec4<T> rv = FIRST ? *(const Vec4<T>*)(ro + row + h0) : ld_stream4(ro + row + h0);
    T out[4];
    if (FIRST) {
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = -scale * rv.v[q] * inv_diag;
    } else {
      const int kp = (k + 1) & m, km = (k - 1) & m;
      const Vec4<T> xc = *(const Vec4<T>*)(ex + row + h0);
      const Vec4<T> ym = *(const Vec4<T>*)(ex + ((int64_t)k * n + jm) * hn + h0);
      const Vec4<T> yp = *(const Vec4<T>*)(ex + ((int64_t)k * n + jp) * hn + h0);
      const Vec4<T> zm = *(const Vec4<T>*)(ex + ((int64_t)km * n + j) * hn + h0);
      const Vec4<T> zp = *(const Vec4<T>*)(ex + ((int64_t)kp * n + j) * hn + h0);
      // x neighbours i -+ 1 sit at half index h - 1 + p and h + p; the one
      // outside the vector: cell 2 h0 - 1 (p = 0) or 2 h0 + 8 (p = 1), read
      // from memory (taking it from the neighbour lane, as the residual
      // kernels do, measured no faster here)
      const T xs = ex[row + ((p ? (2 * h0 + 8) : (2 * h0 - 1)) & m) / 2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T xl = p ? xc.v[q] : (q == 0 ? xs : xc.v[q - 1]);
        const T xr = p ? (q == 3 ? xs : xc.v[q + 1]) : xc.v[q];
        out[q] = (xl + xr + ym.v[q] + yp.v[q] + zm.v[q] + zp.v[q] - scale * rv.v[q]) * inv_diag;
      }
    }
    if (2 * h0 + p >= b.lo[0] && 2 * h0 + 6 + p <= b.hi[0]) {
      Vec4<T> o;
#pragma unroll
      for (int q = 0; q < 4; ++q) o.v[q] = out[q];
      if (FIRST)
        *(Vec4<T>*)(eo + row + h0) = o;
      else
        st_stream4(eo + row + h0, o);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 2 * (h0 + q) + p;
        if (i >= b.lo[0] && i <= b.hi[0]) eo[row + h0 + q] = out[q];
      }
    }
  }
}

// Four colour sweeps (red, black, red, black) of a periodic FP32 level in
// one pass, with the arithmetic of four k_smooth_color_v4 launches (same
// operands, same order: bit-identical results).  Four separate sweeps move
// 24 bytes per cell (each half sweep reads the other colour and its own r,
// writes its own colour); here each cell's r and input black value are read
// once and its final red and black values written once: 10 bytes per cell
// (8 with the zero initial guess, which reads no e).
//
// Each workgroup marches the planes of one column of the mesh: 8 UX cells in
// x by TY rows, zc planes, widened by a halo of 8 cells in x and 4 rows in y
// that the neighbouring columns also compute (sweep s needs sweep s - 1 one
// cell further out, so the valid region shrinks by one cell per sweep).
// Wide columns pay: a region row starts and ends 16 bytes into the cache
// lines of the neighbouring columns, whose reads hit in L2 only as far as
// the columns keep pace with each other (512^3: 128 x 32-cell columns,
// 0.31 ms per pass, against 0.41 ms for 64 x 32 and 0.36 ms for 64 x 64).  In
// step z the four sweeps work on planes z, z - 1, z - 2, z - 3 (each sweep
// needs the previous one on its plane and the two planes next to it), with
// a workgroup barrier between sweeps; their planes live in LDS rings of 6
// planes per colour.  A chunk of zc planes takes zc + 6 steps (three planes
// of warm-up on each side are recomputed by the chunks below and above).
//
// Thread t owns region unit t: 4 half-row entries of one row (8 cells in x,
// both colours) in every sweep, so r and the input black values of its unit
// are prefetched into register queues indexed by plane mod 6 (r 3 steps
// ahead, black e 6 steps ahead); the step loop is unrolled by 6, so that
// queue entries and LDS slots are compile-time constants.  r is read with
// ordinary (cached) loads: the neighbouring columns read the same halo
// lines, and the non-temporal hint cost those hits (512^3: 0.51 -> 0.42 ms
// per pass).  The outputs go out through buffer
// stores that every lane issues in every step, with an offset past the
// plane for lanes or steps without output (dropped by the hardware), so
// that the number of memory operations per step is fixed and the compiler's
// waits for the prefetched loads count exactly.
//
// RES (pre-smoothing): a fifth stage forms the red residual t = r - A e of
// the result (the arithmetic of k_resid_red_v4) one plane behind the last
// sweep and writes it to tout's red half instead of writing the red result
// (which nothing reads before the post-smoothing sets it anew): the black
// ring keeps one more plane (7), the halo one more row, and the first
// sweep takes the black input just outside the region in x from ldsx.
//
// Requires n a power of two >= 8 UX, n % zc == 0.  FIRST: the red sweep starts
// from e = 0 and ein is not read (eout may be the level's e); otherwise ein
// supplies the black colour and must not alias eout (other workgroups still
// read the input halo while this one writes).
template <int V>
struct StepPhase {
  static constexpr int value = V;
};

template <bool FIRST, bool RES, bool BOX, int UX, int TY, int NT>
__global__ void __launch_bounds__(NT)
k_sweep4(const float* __restrict__ ein, float* __restrict__ eout, const float* __restrict__ r, int n,
         int zc, float scale, float inv_diag, float* __restrict__ tout, float inv_scale, float kappa,
         Box b) {
  constexpr int G = RES ? 1 : 0;                 // the residual: one more stage
  constexpr int HY = 4 + G;                      // halo rows per side
  constexpr int U = UX + 2, HW = 4 * U, RY = TY + 2 * HY, PL = RY * HW;   // region: U units x RY rows
  constexpr int ITEMS = RY * U;
  static_assert(ITEMS <= NT, "one region unit per thread");
  constexpr int L = 6, NS = 6, NB = NS + G, D = L - 3;   // queue length = unroll = red LDS slots
  __shared__ __align__(16) float ldsb[NB * PL];
  __shared__ __align__(16) float ldsr[NS * PL];
  __shared__ float ldsx[RES ? NB * 2 * RY : 1];   // black input just outside the region in x
  const int hn = n >> 1, m = n - 1, hm = hn - 1;
  const int64_t oth = (int64_t)n * n * hn, pls = (int64_t)n * hn;
  // columns over the mesh, or with BOX over the box (from its first
  // 4-aligned half index, row and plane)
  const int hb = BOX ? ((b.lo[0] >> 1) & ~3) : 0;
  const Tile tl = BOX ? tile_of(((b.hi[0] >> 1) - hb + 4 * UX) / (4 * UX), (b.hi[1] - b.lo[1] + TY) / TY)
                      : tile_of(n / (8 * UX), n / TY);
  const int H0 = hb + tl.bx * 4 * UX, Y0 = (BOX ? b.lo[1] : 0) + tl.by * TY;
  const int Z0 = (BOX ? b.lo[2] : 0) + tl.bz * zc;
  const int zend = BOX ? min(Z0 + zc, b.hi[2] + 1) : Z0 + zc;   // output planes [Z0, zend)
  const int tid = threadIdx.x;
  const bool ok = tid < ITEMS;
  const int y = ok ? tid / U : 0, u = ok ? tid % U : 0;
  const int jj = (Y0 - HY + y) & m;
  // with BOX every value outside the box is 0 (homogeneous Dirichlet
  // correction): staged inputs and computed values are masked per cell, by
  // the unwrapped coordinates (the box keeps one plane from the mesh's
  // faces, so a wrapped index always lies outside it)
  const int hu = H0 - 4 + 4 * u, ju = Y0 - HY + y;
  const bool rowin = !BOX || (ju >= b.lo[1] && ju <= b.hi[1]);
  auto mask = [&](int c, int z, int h, Vec4<float>& v) {
    if constexpr (BOX) {
      const bool in = rowin && z >= b.lo[2] && z <= b.hi[2];
      const int p = (c + jj + (z & m)) & 1;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int x = 2 * (h + w) + p;
        if (!(in && x >= b.lo[0] && x <= b.hi[0])) v.v[w] = 0.f;
      }
    }
  };
  auto mask1 = [&](int c, int z, int h, float& v) {   // one entry at half index h
    if constexpr (BOX) {
      const int x = 2 * h + ((c + jj + (z & m)) & 1);
      if (!(rowin && z >= b.lo[2] && z <= b.hi[2] && x >= b.lo[0] && x <= b.hi[0])) v = 0.f;
    }
  };
  const int jh = jj * hn + ((H0 - 4 + 4 * u) & hm);   // row and half index of the unit
  const int base = 4 * tid;                            // its place in an LDS plane
  // the other colour's entry next to the unit (clamped to the region: at
  // its edge the value only feeds halo cells that no output depends on;
  // with RES the first sweep takes the true values there instead, from
  // ldsx, since the residual needs one cell more)
  const int xlo = y * HW + max(4 * u - 1, 0);
  const int xhi = y * HW + min(4 * u + 4, HW - 1);
  const bool edge_l = u == 0, edge_r = u == U - 1;
  const int jx = jj * hn + (edge_r ? ((H0 - 4 + 4 * U) & hm) : ((H0 - 5) & hm));
  // output units: the column's, and with BOX only those in the box's rows
  // and overlapping its x range (others would wrap onto cells of the box)
  const bool outp = y >= HY && y < HY + TY && u >= 1 && u <= UX &&
                    (!BOX || (rowin && hu + 3 >= (b.lo[0] >> 1) && hu <= (b.hi[0] >> 1)));
  // plane z of the black ring in slot (z - Z0 + 24) mod 6, with RES
  // (z - Z0 + 28) mod 7 (one more plane: the residual's)
  auto bs = [&](int z) { return ldsb + ((z - Z0 + (RES ? 28 : 24)) % NB) * PL; };
  auto xs_of = [&](int z) { return ldsx + ((z - Z0 + 28) % NB) * 2 * RY; };
  // red r of plane P in qr[(P - zs) mod L], black r in qb, input black e in
  // qe (and its value outside the region in qx); with RES the residual's r,
  // red result and the black results of the two planes next to it in q5r,
  // q3, q4 (indexed by plane mod 3)
  Vec4<float> qr[L], qb[L], qe[L];
  float qx[RES ? L : 1];
  Vec4<float> q5r[RES ? 3 : 1], q3[RES ? 3 : 1], q4[RES ? 3 : 1];
  const int zs = Z0 - 3 - G, ze = Z0 + zc + 2 + G;
  auto ld_r = [&](int c, int z) { return *(const Vec4<float>*)(r + c * oth + (int64_t)(z & m) * pls + jh); };
  auto ld_e = [&](int z) { return *(const Vec4<float>*)(ein + oth + (int64_t)(z & m) * pls + jh); };
  auto ld_x = [&](int z) { return ein[oth + (int64_t)(z & m) * pls + jx]; };
  // colour c on plane z, rows [lo, RY - lo): s* = the other colour's planes
  // z - 1, z, z + 1; the result goes to ov and (keep) to dst
  auto sweep = [&](int c, int z, const float* sm, const float* s0, const float* sp, float* dst, int lo,
                   bool zero, const Vec4<float>& rv, bool keep, Vec4<float>& ov, const float* sx) {
    if (!ok || y < lo || y >= RY - lo) return;
    const int p = (c + jj + (z & m)) & 1;   // cell q of the unit: x = 2 (h0 + q) + p
    if (zero) {
#pragma unroll
      for (int w = 0; w < 4; ++w) ov.v[w] = -scale * rv.v[w] * inv_diag;
    } else {
      const Vec4<float> xc = *(const Vec4<float>*)(s0 + base);
      const Vec4<float> ym = *(const Vec4<float>*)(s0 + base - HW);
      const Vec4<float> yp = *(const Vec4<float>*)(s0 + base + HW);
      const Vec4<float> zm = *(const Vec4<float>*)(sm + base);
      const Vec4<float> zp = *(const Vec4<float>*)(sp + base);
      float xs = s0[p ? xhi : xlo];
      if (sx && (p ? edge_r : edge_l)) xs = sx[(p ? RY : 0) + y];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        // x neighbours: xc[w] and the one on the p side, in this order
        // (k_smooth_color_v4 adds them the other way round for p = 0; the
        // sum of two floats does not depend on the order)
        const float side = p ? (w == 3 ? xs : xc.v[w + 1]) : (w == 0 ? xs : xc.v[w - 1]);
        ov.v[w] = (xc.v[w] + side + ym.v[w] + yp.v[w] + zm.v[w] + zp.v[w] - scale * rv.v[w]) * inv_diag;
      }
    }
    mask(c, z, hu, ov);
    if (keep) *(Vec4<float>*)(dst + base) = ov;
  };
  // red residual t = r - A e on plane z (rows [HY, RY - HY)) with the
  // arithmetic of k_resid_red_v4: black neighbours in the plane from s0, in
  // the planes next to it from bm / bp, the cell's red value ctr
  auto resid = [&](int z, const float* s0, const Vec4<float>& bm, const Vec4<float>& bp,
                   const Vec4<float>& ctr, const Vec4<float>& rv, Vec4<float>& ov) {
    if (!ok || y < HY || y >= RY - HY) return;
    const int p = (jj + (z & m)) & 1;
    const Vec4<float> xc = *(const Vec4<float>*)(s0 + base);
    const Vec4<float> ym = *(const Vec4<float>*)(s0 + base - HW);
    const Vec4<float> yp = *(const Vec4<float>*)(s0 + base + HW);
    const float xs = s0[p ? xhi : xlo];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const float side = p ? (w == 3 ? xs : xc.v[w + 1]) : (w == 0 ? xs : xc.v[w - 1]);
      const float nb = xc.v[w] + side + ym.v[w] + yp.v[w] + bm.v[w] + bp.v[w];
      ov.v[w] = rv.v[w] - (nb - 6.0f * ctr.v[w]) * inv_scale + kappa * ctr.v[w];
    }
    mask(0, z, hu, ov);
  };
  auto put = [&](float* dst, int c, int z, bool valid, const Vec4<float>& ov) {
    const __amdgpu_buffer_rsrc_t rsc = __builtin_amdgcn_make_buffer_rsrc(
        dst + c * oth + (int64_t)(z & m) * pls, (short)0, (int)(pls * 4), 0x00020000);
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f d;
    d.x = ov.v[0], d.y = ov.v[1], d.z = ov.v[2], d.w = ov.v[3];
    const unsigned off = (valid && outp) ? (unsigned)jh * 4u : 0x80000000u;
    __builtin_amdgcn_raw_buffer_store_b128(d, rsc, off, 0, 2 /* non-temporal */);
  };
  auto stage_black = [&](int z, Vec4<float> v, float vx) {
    if (!ok) return;
    mask(1, z, hu, v);
    *(Vec4<float>*)(bs(z) + base) = v;
    if (RES && (edge_l || edge_r)) {
      mask1(1, z, edge_r ? H0 - 4 + 4 * U : H0 - 5, vx);
      xs_of(z)[(edge_r ? RY : 0) + y] = vx;
    }
  };
  // input black planes zs - 1 .. zs + 1 into LDS; queues: red r planes
  // zs - 2 .. zs + D - 1, black r planes zs - 3 .. zs + D - 2, black e
  // planes zs + 2 .. zs + L + 1 (all in bounds: plane indices wrap)
  if (!FIRST) {
    for (int z = zs - 1; z <= zs + 1; ++z) stage_black(z, ld_e(z), RES ? ld_x(z) : 0.f);
  }
#pragma unroll
  for (int x = -2; x < D; ++x) qr[(x + L) % L] = ld_r(0, zs + x);
#pragma unroll
  for (int x = -3; x < D - 1; ++x) qb[(x + L) % L] = ld_r(1, zs + x);
  if (!FIRST) {
#pragma unroll
    for (int x = 2; x < L + 2; ++x) {
      qe[x % L] = ld_e(zs + x);
      if constexpr (RES) qx[x % L] = ld_x(zs + x);
    }
  }
  __syncthreads();
  auto step = [&](int z, auto ph) {
    constexpr int P = decltype(ph)::value;   // z = zs + P (mod 6)
    // black slots (compile-time without RES: plane z + X in (P + X + 3) mod 6)
    auto B = [&](auto x) {
      if constexpr (RES) return bs(z + decltype(x)::value);
      else return ldsb + ((P + decltype(x)::value + 3 + NS) % NS) * PL;
    };
    auto R = [&](auto x) { return ldsr + ((P + decltype(x)::value + 3 + G + NS) % NS) * PL; };
    using M4 = StepPhase<-4>;
    using M3 = StepPhase<-3>;
    using M2 = StepPhase<-2>;
    using M1 = StepPhase<-1>;
    using Z = StepPhase<0>;
    using P1 = StepPhase<1>;
    using P2 = StepPhase<2>;
    // the black input of plane z + 2: into its slot now, or with RES at the
    // end of the step (its slot holds the residual's plane until then)
    Vec4<float> hold;
    float holdx = 0.f;
    if (!FIRST) {
      hold = qe[(P + 2) % L];
      if constexpr (RES) holdx = qx[(P + 2) % L];
      if (!RES && ok && z <= ze) {
        Vec4<float> v = hold;
        mask(1, z + 2, hu, v);
        *(Vec4<float>*)(B(P2{}) + base) = v;
      }
      qe[(P + 2) % L] = ld_e(z + 2 + L);
      if constexpr (RES) qx[(P + 2) % L] = ld_x(z + 2 + L);
    }
    if constexpr (RES) q5r[P % 3] = qr[(P - 2 + L) % L];   // red r of plane z - 2, for step z + 2
    qr[(P + D) % L] = ld_r(0, z + D);
    qb[(P + D - 1 + L) % L] = ld_r(1, z - 1 + D);
    Vec4<float> o1, o2, o3, o4, o5;
    // sweep k (k = 1..4) on plane z - k + 1 for planes in
    // [Z0 - 4 - G + k, Z0 + zc + 3 + G - k]
    if (z <= ze) sweep(0, z, B(M1{}), B(Z{}), B(P1{}), R(Z{}), 1, FIRST, qr[P % L], true, o1,
                       RES && !FIRST ? xs_of(z) : nullptr);
    __syncthreads();
    if (z - 1 >= Z0 - 2 - G && z - 1 <= ze - 1)
      sweep(1, z - 1, R(M2{}), R(M1{}), R(Z{}), B(M1{}), 2, false, qb[(P - 1 + L) % L], true, o2,
            nullptr);
    __syncthreads();
    if (z - 2 >= Z0 - 1 - G && z - 2 <= ze - 2)
      sweep(0, z - 2, B(M3{}), B(M2{}), B(M1{}), R(M2{}), 3, false, qr[(P - 2 + L) % L], true, o3,
            nullptr);
    if constexpr (RES) q3[P % 3] = o3;   // red result of plane z - 2, for the residual at step z + 2
    else put(eout, 0, z - 2, z - 2 >= Z0 && z - 2 < zend, o3);
    __syncthreads();
    if (z - 3 >= Z0 - G && z - 3 <= ze - 3)
      sweep(1, z - 3, R(M4{}), R(M3{}), R(M2{}), B(M3{}), 4, false, qb[(P - 3 + L) % L], RES, o4,
            nullptr);
    put(eout, 1, z - 3, z - 3 >= Z0 && z - 3 < zend, o4);
    if constexpr (RES) {
      // red residual of plane z - 4: black results of planes z - 5 (q4,
      // two steps ago) and z - 3 (o4), red result and r of plane z - 4
      const bool vr = z - 4 >= Z0 && z - 4 < zend;
      if (vr) resid(z - 4, B(M4{}), q4[(P + 1) % 3], o4, q3[(P + 1) % 3], q5r[(P + 1) % 3], o5);
      put(tout, 0, z - 4, vr, o5);
      q4[P % 3] = o4;
      if (!FIRST && z <= ze) stage_black(z + 2, hold, holdx);
    }
    __syncthreads();
  };
  // whole groups of 6 steps (steps past ze only load)
  for (int z = zs; z <= ze; z += L) {
    step(z, StepPhase<0>{});
    step(z + 1, StepPhase<1>{});
    step(z + 2, StepPhase<2>{});
    step(z + 3, StepPhase<3>{});
    step(z + 4, StepPhase<4>{});
    step(z + 5, StepPhase<5>{});
  }
}

// k_resid_red with 4 red cells per thread (see k_smooth_color_v4).
template <typename T, int TXV>
__global__ void __launch_bounds__(256)
k_resid_red_v4(const T* __restrict__ e, const T* __restrict__ r, T* __restrict__ tout, int n, Box b,
               T inv_scale, T kappa) {
  constexpr int TY = 256 / TXV;
  const int hb = (b.lo[0] >> 1) & ~3, hhi = b.hi[0] >> 1;
  const Tile tl = tile_of((hhi - hb + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  const int h0 = hb + (tl.bx * TXV + threadIdx.x) * 4;
  if (j > b.hi[1] || h0 > hhi) return;
  const int m = n - 1, hn = n >> 1;
  const int64_t oth = half_cells(n);
  const int k0 = b.lo[2] + tl.bz * kVecKz;
  const int k1 = min(k0 + kVecKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m;
  const bool lane_l = threadIdx.x > 0, lane_r = threadIdx.x + 1 < TXV && h0 + 4 <= hhi;
  for (int k = k0; k <= k1; ++k) {
    const int p = (j + k) & 1;
    const int kp = (k + 1) & m, km = (k - 1) & m;
    const int64_t row = ((int64_t)k * n + j) * hn;
    const Vec4<T> ctr = ld_stream4(e + row + h0);
    const Vec4<T> rv = ld_stream4(r + row + h0);
    const Vec4<T> xc = *(const Vec4<T>*)(e + oth + row + h0);
    const Vec4<T> ym = *(const Vec4<T>*)(e + oth + ((int64_t)k * n + jm) * hn + h0);
    const Vec4<T> yp = *(const Vec4<T>*)(e + oth + ((int64_t)k * n + jp) * hn + h0);
    const Vec4<T> zm = *(const Vec4<T>*)(e + oth + ((int64_t)km * n + j) * hn + h0);
    const Vec4<T> zp = *(const Vec4<T>*)(e + oth + ((int64_t)kp * n + j) * hn + h0);
    const T sl = lane_prev<TXV>(xc.v[3]), sr = lane_next<TXV>(xc.v[0]);
    T xs = p ? sr : sl;
    if (p ? !lane_r : !lane_l) xs = e[oth + row + ((p ? (2 * h0 + 8) : (2 * h0 - 1)) & m) / 2];
    T out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T xl = p ? xc.v[q] : (q == 0 ? xs : xc.v[q - 1]);
      const T xr = p ? (q == 3 ? xs : xc.v[q + 1]) : xc.v[q];
      const T nb = xl + xr + ym.v[q] + yp.v[q] + zm.v[q] + zp.v[q];
      out[q] = rv.v[q] - (nb - (T)6 * ctr.v[q]) * inv_scale + kappa * ctr.v[q];
    }
    if (2 * h0 + p >= b.lo[0] && 2 * h0 + 6 + p <= b.hi[0]) {
      Vec4<T> o;
#pragma unroll
      for (int q = 0; q < 4; ++q) o.v[q] = out[q];
      *(Vec4<T>*)(tout + row + h0) = o;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 2 * (h0 + q) + p;
        if (i >= b.lo[0] && i <= b.hi[0]) tout[row + h0 + q] = out[q];
      }
    }
  }
}

// t = r - A_l e on the red cells of the box.  After a sweep that ends with
// the black colour the black residual is zero (each black equation was just
// solved exactly), so t keeps zeros there (t is cleared with the levels).
template <typename T>
__global__ void __launch_bounds__(256)
k_resid_red(const T* __restrict__ e, const T* __restrict__ r, T* __restrict__ tout, int n, Box b,
            T inv_scale, T kappa) {
  const Tile tl = tile_half(b);
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (j > b.hi[1]) return;
  const int h = (b.lo[0] >> 1) + tl.bx * kBoxTx + threadIdx.x;
  const int m = n - 1, hn = n >> 1;
  const int64_t oth = half_cells(n);
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m;
  for (int k = k0; k <= k1; ++k) {
    const int i = 2 * h + ((j + k) & 1);
    if (i < b.lo[0] || i > b.hi[0]) continue;
    const int kp = (k + 1) & m, km = (k - 1) & m;
    const int64_t row = ((int64_t)k * n + j) * hn;
    const int64_t c = row + h;
    const T ctr = e[c];
    const T nb = e[oth + row + (((i - 1) & m) >> 1)] + e[oth + row + (((i + 1) & m) >> 1)] +
                 e[oth + ((int64_t)k * n + jm) * hn + h] + e[oth + ((int64_t)k * n + jp) * hn + h] +
                 e[oth + ((int64_t)km * n + j) * hn + h] + e[oth + ((int64_t)kp * n + j) * hn + h];
    tout[c] = r[c] - (nb - (T)6 * ctr) * inv_scale + kappa * ctr;
  }
}

// Full weighting: r_c(I) = sum_{o in {-1,0,1}^3} w(o) t_f(2I + o),
// w = (1/4, 1/2, 1/4) per axis.  Only red fine cells (o_x + o_y + o_z even)
// carry a residual.
template <typename T>
__global__ void __launch_bounds__(256)
k_restrict(const T* __restrict__ tf, T* __restrict__ rc, int nf, int nc, Box bc) {
  const Tile tl = tile_box(bc);
  const int I = bc.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int J = bc.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (I > bc.hi[0] || J > bc.hi[1]) return;
  const int m = nf - 1;
  const int K0 = bc.lo[2] + tl.bz * kBoxKz;
  const int K1 = min(K0 + kBoxKz - 1, bc.hi[2]);
  const int hn = nf >> 1;
  for (int K = K0; K <= K1; ++K) {
    // red fine cells of the 3x3x3 stencil, grouped by weight
    const int i = 2 * I, j = 2 * J, k = 2 * K;
    const int im = (i - 1) & m, ip = (i + 1) & m, jm = (j - 1) & m, jp = (j + 1) & m;
    const int km = (k - 1) & m, kp = (k + 1) & m;
    auto R = [&](int x, int y, int z) -> T { return tf[((int64_t)z * nf + y) * hn + (x >> 1)]; };
    const T centre = R(i, j, k);
    const T edges = R(im, jm, k) + R(ip, jm, k) + R(im, jp, k) + R(ip, jp, k) +
                    R(im, j, km) + R(ip, j, km) + R(im, j, kp) + R(ip, j, kp) +
                    R(i, jm, km) + R(i, jp, km) + R(i, jm, kp) + R(i, jp, kp);
    rc[sidx(I, J, K, nc)] = (T)0.125 * centre + (T)0.03125 * edges;
  }
}

// Prolongation and correction of the black cells only: the next sweep starts
// with the red colour, whose update reads only black neighbours and
// overwrites the red values, so red cells need no correction.  Threads map
// to (h, j, k) like the smoother; with all_cells each thread also corrects
// the red cell of its pair.  Trilinear: fine cell i takes the mean of coarse
// cells i >> 1 and (i >> 1) + (i & 1) per axis (they coincide for even i).
// A workgroup's fine tile (2 kBoxTx x kBoxTy x kBoxKz cells) reads coarse
// cells in a (kBoxTx + 1) x 3 x (kBoxKz / 2 + 1) block, staged once in LDS.
constexpr int kPcx = kBoxTx + 1, kPcy = kBoxTy / 2 + 1, kPcz = kBoxKz / 2 + 1;

template <typename T>
__global__ void __launch_bounds__(256)
k_prolong(const T* __restrict__ ec, T* __restrict__ ef, int nc, int nf, Box bf, int all_cells) {
  __shared__ T cs[kPcz][kPcy][kPcx];
  const Tile tl = tile_half(bf);
  const int h0 = (bf.lo[0] >> 1) + tl.bx * kBoxTx;
  const int j0 = bf.lo[1] + tl.by * kBoxTy;
  const int k0 = bf.lo[2] + tl.bz * kBoxKz;
  const int J0 = j0 >> 1, K0 = k0 >> 1, mc = nc - 1;
  const int tid = threadIdx.y * kBoxTx + threadIdx.x;
  for (int q = tid; q < kPcz * kPcy * kPcx; q += 256) {
    const int ii = q % kPcx, jj = (q / kPcx) % kPcy, kk = q / (kPcx * kPcy);
    cs[kk][jj][ii] = ec[sidx((h0 + ii) & mc, (J0 + jj) & mc, (K0 + kk) & mc, nc)];
  }
  __syncthreads();
  const int j = j0 + threadIdx.y;
  if (j > bf.hi[1]) return;
  const int h = h0 + threadIdx.x;
  const int hn = nf >> 1;
  const int64_t hc = half_cells(nf);
  const int k1 = min(k0 + kBoxKz - 1, bf.hi[2]);
  const int y0 = (j >> 1) - J0, y1 = y0 + (j & 1);
  const int x0 = threadIdx.x;
  for (int k = k0; k <= k1; ++k) {
    const int64_t row = ((int64_t)k * nf + j) * hn + h;
    const int z0 = (k >> 1) - K0, z1 = z0 + (k & 1);
    for (int color = all_cells ? 0 : 1; color < 2; ++color) {
      const int i = 2 * h + ((color + j + k) & 1);
      if (i < bf.lo[0] || i > bf.hi[0]) continue;
      const int x1 = x0 + (i & 1);
      const T a = cs[z0][y0][x0] + cs[z0][y0][x1] + cs[z0][y1][x0] + cs[z0][y1][x1] +
                  cs[z1][y0][x0] + cs[z1][y0][x1] + cs[z1][y1][x0] + cs[z1][y1][x1];
      ef[color * hc + row] += (T)0.125 * a;
    }
  }
}

// FP32 forms of the restriction and of the black-cell prolongation with 4
// cells per thread in the tiles of k_smooth_color_v4 (256 threads, TXV
// across a row), so that the fine level is read and written in aligned
// 16-byte vectors.  They need n_fine / 2 and n_coarse / 2 to be multiples of
// 4 and 2 (the host takes them for fine boxes of at least 64 cells a row).
//
// Restriction of 4 coarse cells I0 .. I0 + 3 (I0 a multiple of 4): the red
// fine cells of k_restrict's stencil lie at half index I in the rows whose
// offsets (o_y, o_z) are both even or both odd (the centre and the four
// diagonal rows) and at half indices I - 1 and I in the other four rows, so
// each fine row is one vector (plus the value before it).  The coarse cells
// alternate colours: I0 and I0 + 2 are one aligned pair of one colour's half,
// I0 + 1 and I0 + 3 the pair at the same offset in the other half.
template <int TXV>
__global__ void __launch_bounds__(256)
k_restrict_v4(const float* __restrict__ tf, float* __restrict__ rc, int nf, int nc, Box bc) {
  constexpr int TY = 256 / TXV;
  const int ib = bc.lo[0] & ~3;
  const Tile tl = tile_of((bc.hi[0] - ib + 4 * TXV) / (4 * TXV), (bc.hi[1] - bc.lo[1] + TY) / TY);
  const int J = bc.lo[1] + tl.by * TY + threadIdx.y;
  const int I0 = ib + (tl.bx * TXV + threadIdx.x) * 4;
  if (J > bc.hi[1] || I0 > bc.hi[0]) return;
  const int m = nf - 1, hn = nf >> 1, hnc = nc >> 1;
  const int64_t hcc = half_cells(nc);
  const int K0 = bc.lo[2] + tl.bz * kVecKz;
  const int K1 = min(K0 + kVecKz - 1, bc.hi[2]);
  const int j = 2 * J, jm = (j - 1) & m, jp = (j + 1) & m;
  const int before = (I0 - 1) & (hn - 1);
  for (int K = K0; K <= K1; ++K) {
    const int k = 2 * K, km = (k - 1) & m, kp = (k + 1) & m;
    auto row = [&](int y, int z) { return tf + ((int64_t)z * nf + y) * hn; };
    const Vec4<float> centre = *(const Vec4<float>*)(row(j, k) + I0);
    float edges[4] = {0.f, 0.f, 0.f, 0.f};
    const int pr[4][2] = {{jm, k}, {jp, k}, {j, km}, {j, kp}};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float* rp = row(pr[t][0], pr[t][1]);
      const Vec4<float> v = *(const Vec4<float>*)(rp + I0);
      const float b = rp[before];
#pragma unroll
      for (int q = 0; q < 4; ++q) edges[q] += (q == 0 ? b : v.v[q - 1]) + v.v[q];
    }
    const int dg[4][2] = {{jm, km}, {jp, km}, {jm, kp}, {jp, kp}};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const Vec4<float> v = *(const Vec4<float>*)(row(dg[t][0], dg[t][1]) + I0);
#pragma unroll
      for (int q = 0; q < 4; ++q) edges[q] += v.v[q];
    }
    float out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = 0.125f * centre.v[q] + 0.03125f * edges[q];
    const int s = (J + K) & 1;                  // colour of coarse cell I0
    const int64_t crow = ((int64_t)K * nc + J) * hnc + (I0 >> 1);
    if (I0 >= bc.lo[0] && I0 + 3 <= bc.hi[0]) {
      Vec2<float> a, b;
      a.v[0] = out[0], a.v[1] = out[2];
      b.v[0] = out[1], b.v[1] = out[3];
      *(Vec2<float>*)(rc + s * hcc + crow) = a;
      *(Vec2<float>*)(rc + (s ^ 1) * hcc + crow) = b;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (I0 + q >= bc.lo[0] && I0 + q <= bc.hi[0])
          rc[((s + q) & 1) * hcc + crow + (q >> 1)] = out[q];
    }
  }
}

// Black-cell prolongation (k_prolong without all_cells) for the 4 black
// cells 2 (h0 + q) + p of a fine row: cell q takes coarse x h0 + q and
// h0 + q + p, so the row needs coarse x h0 .. h0 + 4 from each coarse row
// (Y, Z) it draws on: two aligned pairs (one per colour half) and one more
// value.  Rows coinciding with a coarse row (even j or k) are summed once
// and weighted twice.
template <int TXV>
__global__ void __launch_bounds__(256)
k_prolong_black_v4(const float* __restrict__ ec, float* __restrict__ ef, int nc, int nf, Box bf) {
  constexpr int TY = 256 / TXV;
  const int hb = (bf.lo[0] >> 1) & ~3, hhi = bf.hi[0] >> 1;
  const Tile tl = tile_of((hhi - hb + 4 * TXV) / (4 * TXV), (bf.hi[1] - bf.lo[1] + TY) / TY);
  const int j = bf.lo[1] + tl.by * TY + threadIdx.y;
  const int h0 = hb + (tl.bx * TXV + threadIdx.x) * 4;
  if (j > bf.hi[1] || h0 > hhi) return;
  const int mc = nc - 1, hnf = nf >> 1, hnc = nc >> 1;
  const int64_t hcf = half_cells(nf), hcc = half_cells(nc);
  const int k0 = bf.lo[2] + tl.bz * kVecKz;
  const int k1 = min(k0 + kVecKz - 1, bf.hi[2]);
  const int ny = 1 + (j & 1);
  const int Ys[2] = {j >> 1, ((j >> 1) + 1) & mc};
  const int c0 = h0 >> 1;                       // coarse half index of x = h0 (h0 even)
  const int c4 = ((h0 + 4) & mc) >> 1;          // ... of x = h0 + 4 (even, same colour)
  for (int k = k0; k <= k1; ++k) {
    const int p = (1 + j + k) & 1;
    const int nz = 1 + (k & 1);
    const int Zs[2] = {k >> 1, ((k >> 1) + 1) & mc};
    float L[5] = {0.f, 0.f, 0.f, 0.f, 0.f};   // summed coarse rows at x = h0 + q
    for (int zz = 0; zz < nz; ++zz) {
      for (int yy = 0; yy < ny; ++yy) {
        const int Y = Ys[yy], Z = Zs[zz];
        const int s = (Y + Z) & 1;             // colour of coarse x = h0
        const float* crow = ec + ((int64_t)Z * nc + Y) * hnc;
        const Vec2<float> ev = *(const Vec2<float>*)(crow + s * hcc + c0);        // x = h0, h0 + 2
        const Vec2<float> od = *(const Vec2<float>*)(crow + (s ^ 1) * hcc + c0);  // h0 + 1, h0 + 3
        L[0] += ev.v[0];
        L[1] += od.v[0];
        L[2] += ev.v[1];
        L[3] += od.v[1];
        L[4] += crow[s * hcc + c4];
      }
    }
    const float w = 0.125f * (float)((3 - ny) * (3 - nz));
    const int64_t frow = hcf + ((int64_t)k * nf + j) * hnf + h0;
    const Vec4<float> e = ld_stream4(ef + frow);     // read and written once: streamed
    float out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = e.v[q] + w * (L[q] + (p ? L[q + 1] : L[q]));
    if (2 * h0 + p >= bf.lo[0] && 2 * h0 + 6 + p <= bf.hi[0]) {
      Vec4<float> o;
#pragma unroll
      for (int q = 0; q < 4; ++q) o.v[q] = out[q];
      st_stream4(ef + frow, o);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 2 * (h0 + q) + p;
        if (i >= bf.lo[0] && i <= bf.hi[0]) ef[frow + q] = out[q];
      }
    }
  }
}

// Coarsest level: one workgroup; e lives in LDS on a box-local array of at
// most kCoarseMax^3 entries: the whole (periodic) level, or the box plus a
// one-cell ring of zeros (Dirichlet).  Each thread owns up to kCoarseMax^3 /
// 1024 cells whose LDS offsets and right-hand sides stay in registers for all
// `sweeps` red-black sweeps.  With project != 0 (periodic, kappa = 0) the
// mean of r is removed first and the mean of e afterwards.  The host checks
// that the local array fits.
constexpr int kCoarsePer = kCoarseMax * kCoarseMax * kCoarseMax / 1024;

template <typename T>
__global__ void __launch_bounds__(1024)
k_coarse(T* __restrict__ e, const T* __restrict__ r, int n, Box b, T scale, T inv_diag,
         int sweeps, int project, int periodic) {
  __shared__ T es[kCoarseMax * kCoarseMax * kCoarseMax];
  __shared__ double sh[16];
  const int tid = threadIdx.x;
  const int nx = b.hi[0] - b.lo[0] + 1, ny = b.hi[1] - b.lo[1] + 1, nz = b.hi[2] - b.lo[2] + 1;
  const int nbox = nx * ny * nz;
  const int off = periodic ? 0 : 1;
  const int lx = nx + 2 * off, ly = ny + 2 * off, lz = nz + 2 * off;
  const int m = n - 1;
  for (int c = tid; c < lx * ly * lz; c += 1024) es[c] = 0;
  // owned cells: local offset of the cell and of its 6 neighbours, colour, rhs
  int own[kCoarsePer], nbr[kCoarsePer][6], col[kCoarsePer];
  T rr[kCoarsePer];
  int64_t gidx[kCoarsePer];
  int nown = 0;
  double racc = 0.0;
#pragma unroll
  for (int u = 0; u < kCoarsePer; ++u) {
    const int q = tid + 1024 * u;
    if (q >= nbox) break;
    nown = u + 1;
    const int qa = q % nx, qb = (q / nx) % ny, qc = q / (nx * ny);
    const int a0 = qa + off, b0 = qb + off, c0 = qc + off;
    int am, ap, bm, bp, cm, cp;
    if (periodic) {
      am = (a0 - 1) & m; ap = (a0 + 1) & m;
      bm = (b0 - 1) & m; bp = (b0 + 1) & m;
      cm = (c0 - 1) & m; cp = (c0 + 1) & m;
    } else {
      am = a0 - 1; ap = a0 + 1; bm = b0 - 1; bp = b0 + 1; cm = c0 - 1; cp = c0 + 1;
    }
    own[u] = (c0 * ly + b0) * lx + a0;
    nbr[u][0] = (c0 * ly + b0) * lx + am;
    nbr[u][1] = (c0 * ly + b0) * lx + ap;
    nbr[u][2] = (c0 * ly + bm) * lx + a0;
    nbr[u][3] = (c0 * ly + bp) * lx + a0;
    nbr[u][4] = (cm * ly + b0) * lx + a0;
    nbr[u][5] = (cp * ly + b0) * lx + a0;
    const int i = b.lo[0] + qa, j = b.lo[1] + qb, k = b.lo[2] + qc;
    col[u] = (i + j + k) & 1;
    gidx[u] = sidx(i, j, k, n);
    rr[u] = r[gidx[u]];
    racc += (double)rr[u];
  }
  if (project) {
    const double s = block_sum<1024>(racc, sh);
    if (tid == 0) sh[8] = s / nbox;
    __syncthreads();
    const T rm = (T)sh[8];
#pragma unroll
    for (int u = 0; u < kCoarsePer; ++u)
      if (u < nown) rr[u] -= rm;
  }
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int color = 0; color < 2; ++color) {
#pragma unroll
      for (int u = 0; u < kCoarsePer; ++u) {
        if (u >= nown || col[u] != color) continue;
        const T nb = es[nbr[u][0]] + es[nbr[u][1]] + es[nbr[u][2]] + es[nbr[u][3]] +
                     es[nbr[u][4]] + es[nbr[u][5]];
        es[own[u]] = (nb - scale * rr[u]) * inv_diag;
      }
      __syncthreads();
    }
  }
  T emean = 0;
  if (project) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kCoarsePer; ++u)
      if (u < nown) acc += (double)es[own[u]];
    const double s = block_sum<1024>(acc, sh);
    if (tid == 0) sh[8] = s / nbox;
    __syncthreads();
    emean = (T)sh[8];
  }
#pragma unroll
  for (int u = 0; u < kCoarsePer; ++u)
    if (u < nown) e[gidx[u]] = es[own[u]] - emean;
}

// Residual of phi + scale * d, with d applied only inside the box (the
// learned initial guess); written colour-split like k_residual.
template <typename T>
__global__ void __launch_bounds__(256)
k_residual_guess(const double* __restrict__ phi, const float* __restrict__ d, double scale,
                 const double* __restrict__ rhs, T* __restrict__ rout, int n, Box b, double kappa,
                 double* __restrict__ partial) {
  __shared__ double sh[4];
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  const int m = n - 1;
  auto inb = [&](int x, int y, int z) {
    return x >= b.lo[0] && x <= b.hi[0] && y >= b.lo[1] && y <= b.hi[1] && z >= b.lo[2] &&
           z <= b.hi[2];
  };
  auto v = [&](int x, int y, int z) -> double {
    const int64_t c = lin(x, y, z, n);
    return inb(x, y, z) ? phi[c] + scale * (double)d[c] : phi[c];
  };
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    const int ip = (i + 1) & m, im = (i - 1) & m, jp = (j + 1) & m, jm = (j - 1) & m;
    for (int k = k0; k <= k1; ++k) {
      const int kp = (k + 1) & m, km = (k - 1) & m;
      const double ctr = v(i, j, k);
      const double nb = v(ip, j, k) + v(im, j, k) + v(i, jp, k) + v(i, jm, k) + v(i, j, kp) +
                        v(i, j, km);
      const double res = rhs[lin(i, j, k, n)] - (nb - 6.0 * ctr - kappa * ctr);
      rout[sidx(i, j, k, n)] = (T)res;
      acc += res * res;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// phi += scale d (and chg += the same increment when given).
__global__ void __launch_bounds__(256)
k_apply_guess(double* __restrict__ phi, const float* __restrict__ d, double scale,
              float* __restrict__ chg, int n, Box b) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    const double inc = scale * (double)d[c];
    phi[c] += inc;
    if (chg) chg[c] += (float)inc;
  }
}

__global__ void __launch_bounds__(256)
k_sum_sq(const double* __restrict__ phi, int n, Box b, double* __restrict__ partial) {
  __shared__ double sh[4];
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + tl.bz * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    for (int k = k0; k <= k1; ++k) {
      const double v = phi[lin(i, j, k, n)];
      acc += v * v;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// Solve recording (training pairs): rec = [r0 | phi_old | dphi], each n^3
// FP32 in natural order; r0 is zero outside the box, dphi starts at zero.
template <typename T>
__global__ void __launch_bounds__(256)
k_record_start(const T* __restrict__ r, const double* __restrict__ phi, int n, Box b,
               float* __restrict__ rec) {
  const int64_t V = (int64_t)n * n * n;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= V) return;
  const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
  const bool in = i >= b.lo[0] && i <= b.hi[0] && j >= b.lo[1] && j <= b.hi[1] && k >= b.lo[2] &&
                  k <= b.hi[2];
  rec[v] = in ? (float)r[sidx(i, j, k, n)] : 0.f;
  rec[V + v] = (float)phi[v];
  rec[2 * V + v] = 0.f;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_record_accum(const T* __restrict__ e, int n, Box b, float* __restrict__ dphi) {
  const Tile tl = tile_box(b);
  const int i = b.lo[0] + tl.bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + tl.by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) dphi[lin(i, j, k, n)] += (float)e[sidx(i, j, k, n)];
}

}  // namespace

// ------------------------------------------------------------- launchers
template <typename T>
void launch_fill(T* a, int n, const Box& b, T v, hipStream_t st) {
  prof_begin(st, K_FILL);
  hipLaunchKernelGGL(k_fill<T>, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, a, n, b, v);
  prof_end(st, K_FILL, (double)box_cells(b) * sizeof(T));
}
template void launch_fill<float>(float*, int, const Box&, float, hipStream_t);
template void launch_fill<double>(double*, int, const Box&, double, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, int, const Box&, uint64_t, hipStream_t);

void launch_rhs(const uint64_t* counts, double* phi, double* rhs, int n, const Box& b,
                double c_scale, double c_off, double kappa, float* chg, double chg_scale,
                bool apply, double* partial, int* nblocks, hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)(g.x * g.y * g.z);
  prof_begin(st, K_RHS);
  if (chg)
    hipLaunchKernelGGL(k_rhs<true>, g, dim3(kBoxTx, kBoxTy), 0, st, counts, phi, rhs, n, b,
                       c_scale, c_off, kappa, chg, chg_scale, apply ? 1 : 0, partial);
  else
    hipLaunchKernelGGL(k_rhs<false>, g, dim3(kBoxTx, kBoxTy), 0, st, counts, phi, rhs, n, b,
                       c_scale, c_off, kappa, nullptr, 0.0, 0, partial);
  prof_end(st, K_RHS, (24.0 + (chg ? (apply ? 16.0 : 4.0) : 0.0)) * box_cells(b));
}

// Threads across a tile row (64, 32 or 16, 4 entries each) for a row of
// `ext` entries: the width that maximises the share of lanes holding row
// entries (the last tile of a row is partly empty) times the rate each width
// reaches on full rows (measured on the 512^3 finest level: 4.77, 4.38 and
// 4.07 TB/s for 64, 32 and 16 threads), so that a box row of 190 entries
// takes three 64-entry tiles rather than two of 128.
inline int tile_threads(int ext) {
  const int widths[3] = {64, 32, 16};
  const double rate[3] = {1.0, 0.92, 0.85};
  int best = 16;
  double score = -1.0;
  for (int q = 0; q < 3; ++q) {
    const int w = 4 * widths[q];
    const double s = (double)ext / (double)(((ext + w - 1) / w) * w) * rate[q];
    if (s > score) {
      score = s;
      best = widths[q];
    }
  }
  return best;
}

template <typename T>
void launch_residual(const double* phi, const double* rhs, T* r_out, int n, const Box& b,
                     double kappa, double* partial, int* nblocks, hipStream_t st) {
  const int ib = b.lo[0] & ~3;
  prof_begin(st, K_RESIDUAL);
  if (b.hi[0] - ib + 1 >= 64) {
    // tile width as for the colour sweeps (the extent here in cells, 4 per thread)
    const int txv = tile_threads(b.hi[0] - ib + 1);
    const unsigned gx = (unsigned)((b.hi[0] - ib + 4 * txv) / (4 * txv));
    const unsigned gy = (unsigned)((b.hi[1] - b.lo[1] + 256 / txv) / (256 / txv));
    const unsigned gz = (unsigned)((b.hi[2] - b.lo[2] + kResKz) / kResKz);
    *nblocks = (int)(gx * gy * gz);
    const dim3 g(gx * gy * gz), blk(txv, 256 / txv);
    if (txv == 64)
      hipLaunchKernelGGL((k_residual_v4<T, 64>), g, blk, 0, st, phi, rhs, r_out, n, b, kappa,
                         partial);
    else if (txv == 32)
      hipLaunchKernelGGL((k_residual_v4<T, 32>), g, blk, 0, st, phi, rhs, r_out, n, b, kappa,
                         partial);
    else
      hipLaunchKernelGGL((k_residual_v4<T, 16>), g, blk, 0, st, phi, rhs, r_out, n, b, kappa,
                         partial);
  } else {
    const dim3 g = box_grid(b);
    *nblocks = (int)(g.x * g.y * g.z);
    hipLaunchKernelGGL(k_residual<T>, g, dim3(kBoxTx, kBoxTy), 0, st, phi, rhs, r_out, n, b, kappa,
                       partial);
  }
  prof_end(st, K_RESIDUAL, (16.0 + sizeof(T)) * box_cells(b));
}
template void launch_residual<float>(const double*, const double*, float*, int, const Box&,
                                     double, double*, int*, hipStream_t);
template void launch_residual<double>(const double*, const double*, double*, int, const Box&,
                                      double, double*, int*, hipStream_t);

// g3 = -(Phi(i+1) - Phi(i-1)) / 2h per axis on the box, 3 FP32 values per
// cell in natural order (the interpolation's one 12-byte load per CIC cell);
// each thread walks kBoxKz planes carrying Phi at k-1 and k.
__global__ void __launch_bounds__(256)
k_force_mesh(const double* __restrict__ phi, float* __restrict__ g3, int n, Box b, double inv2h,
             int gx, int gy) {
  const int64_t bl = xcd_block();
  const int bx = (int)(bl % gx), by = (int)((bl / gx) % gy), bz = (int)(bl / ((int64_t)gx * gy));
  const int i = b.lo[0] + bx * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + by * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int m = n - 1;
  const int k0 = b.lo[2] + bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int ip = (i + 1) & m, im = (i - 1) & m, jp = (j + 1) & m, jm = (j - 1) & m;
  double below = phi[lin(i, j, (k0 - 1) & m, n)], ctr = phi[lin(i, j, k0, n)];
  for (int k = k0; k <= k1; ++k) {
    const double above = phi[lin(i, j, (k + 1) & m, n)];
    float* q = g3 + 3 * lin(i, j, k, n);
    q[0] = (float)(-(phi[lin(ip, j, k, n)] - phi[lin(im, j, k, n)]) * inv2h);
    q[1] = (float)(-(phi[lin(i, jp, k, n)] - phi[lin(i, jm, k, n)]) * inv2h);
    q[2] = (float)(-(above - below) * inv2h);
    below = ctr;
    ctr = above;
  }
}

// k_force_mesh with 4 consecutive cells per thread (tiles as k_residual_v4):
// vector loads of Phi; a lane's 4 cells are 12 contiguous values, so a row
// segment of TXV lanes (always within one wave) is staged in LDS and stored
// as 3 coalesced 16-byte streamed stores per lane (a lane storing its own 48
// bytes leaves each store instruction strided: 0.78 against 0.62 ms at
// 512^3); segments that leave the box store cell by cell.
template <int TXV>
__global__ void __launch_bounds__(256)
k_force_mesh_v4(const double* __restrict__ phi, float* __restrict__ g3, int n, Box b,
                double inv2h) {
  constexpr int TY = 256 / TXV;
  __shared__ __attribute__((aligned(16))) float stage[12 * 256];
  const int ib = b.lo[0] & ~3;
  const Tile tl = tile_of((b.hi[0] - ib + 4 * TXV) / (4 * TXV), (b.hi[1] - b.lo[1] + TY) / TY);
  const int i0 = ib + (tl.bx * TXV + threadIdx.x) * 4;
  const int j = b.lo[1] + tl.by * TY + threadIdx.y;
  if (i0 > b.hi[0] || j > b.hi[1]) return;
  const int m = n - 1;
  const int k0 = b.lo[2] + tl.bz * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m, il = (i0 - 1) & m, ir = (i0 + 4) & m;
  const bool full = i0 >= b.lo[0] && i0 + 3 <= b.hi[0];
  const int seg0 = ib + tl.bx * TXV * 4;          // first cell of this row segment
  const bool row_full = seg0 >= b.lo[0] && seg0 + 4 * TXV - 1 <= b.hi[0];
  const bool lane_l = threadIdx.x > 0, lane_r = threadIdx.x + 1 < TXV && i0 + 4 <= b.hi[0];
  Vec4<double> below = *(const Vec4<double>*)(phi + lin(i0, j, (k0 - 1) & m, n));
  Vec4<double> ctr = *(const Vec4<double>*)(phi + lin(i0, j, k0, n));
  for (int k = k0; k <= k1; ++k) {
    const Vec4<double> above = *(const Vec4<double>*)(phi + lin(i0, j, (k + 1) & m, n));
    const Vec4<double> ym = *(const Vec4<double>*)(phi + lin(i0, jm, k, n));
    const Vec4<double> yp = *(const Vec4<double>*)(phi + lin(i0, jp, k, n));
    double xl = lane_prev<TXV>(ctr.v[3]), xr = lane_next<TXV>(ctr.v[0]);
    if (!lane_l) xl = phi[lin(il, j, k, n)];
    if (!lane_r) xr = phi[lin(ir, j, k, n)];
    float out[12];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double left = q == 0 ? xl : ctr.v[q - 1];
      const double right = q == 3 ? xr : ctr.v[q + 1];
      out[3 * q + 0] = (float)(-(right - left) * inv2h);
      out[3 * q + 1] = (float)(-(yp.v[q] - ym.v[q]) * inv2h);
      out[3 * q + 2] = (float)(-(above.v[q] - below.v[q]) * inv2h);
    }
    float* dst = g3 + 3 * lin(i0, j, k, n);
    if (row_full) {
      // the TXV lanes of a row segment hold 48 TXV contiguous bytes: stage
      // them in LDS and store them back as 3 coalesced 16-byte stores per lane
      float* seg = stage + threadIdx.y * (12 * TXV);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Vec4<float> o;
        o.v[0] = out[4 * v], o.v[1] = out[4 * v + 1], o.v[2] = out[4 * v + 2], o.v[3] = out[4 * v + 3];
        *(Vec4<float>*)(seg + 12 * threadIdx.x + 4 * v) = o;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      float* gseg = g3 + 3 * lin(i0 - 4 * (int)threadIdx.x, j, k, n);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const Vec4<float> o = *(const Vec4<float>*)(seg + 4 * (TXV * v + threadIdx.x));
        st_stream4(gseg + 4 * (TXV * v + threadIdx.x), o);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else if (full) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Vec4<float> o;
        o.v[0] = out[4 * v], o.v[1] = out[4 * v + 1], o.v[2] = out[4 * v + 2], o.v[3] = out[4 * v + 3];
        st_stream4(dst + 4 * v, o);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i0 + q >= b.lo[0] && i0 + q <= b.hi[0])
          for (int d = 0; d < 3; ++d) dst[3 * q + d] = out[3 * q + d];
    }
    below = ctr;
    ctr = above;
  }
}

void launch_force_mesh(const double* phi, float* g3, int n, const Box& b, double inv2h,
                       hipStream_t st) {
  prof_begin(st, K_FORCE_MESH);
  const int ib = b.lo[0] & ~3;
  if (b.hi[0] - ib + 1 >= 64) {
    const int txv = tile_threads(b.hi[0] - ib + 1);
    const unsigned gx = (unsigned)((b.hi[0] - ib + 4 * txv) / (4 * txv));
    const unsigned gy = (unsigned)((b.hi[1] - b.lo[1] + 256 / txv) / (256 / txv));
    const unsigned gz = (unsigned)((b.hi[2] - b.lo[2] + kBoxKz) / kBoxKz);
    const dim3 g(gx * gy * gz), blk(txv, 256 / txv);
    if (txv == 64)
      hipLaunchKernelGGL(k_force_mesh_v4<64>, g, blk, 0, st, phi, g3, n, b, inv2h);
    else if (txv == 32)
      hipLaunchKernelGGL(k_force_mesh_v4<32>, g, blk, 0, st, phi, g3, n, b, inv2h);
    else
      hipLaunchKernelGGL(k_force_mesh_v4<16>, g, blk, 0, st, phi, g3, n, b, inv2h);
  } else {
    const int gx = (b.hi[0] - b.lo[0] + kBoxTx) / kBoxTx, gy = (b.hi[1] - b.lo[1] + kBoxTy) / kBoxTy;
    const int gz = (b.hi[2] - b.lo[2] + kBoxKz) / kBoxKz;
    hipLaunchKernelGGL(k_force_mesh, dim3((unsigned)gx * gy * gz), dim3(kBoxTx, kBoxTy), 0, st,
                       phi, g3, n, b, inv2h, gx, gy);
  }
  prof_end(st, K_FORCE_MESH, 20.0 * box_cells(b));
}

template <typename T>
void launch_correct(double* phi, const T* e, float* chg, double pending_scale, int n,
                    const Box& b, hipStream_t st) {
  prof_begin(st, K_CORRECT);
  if (chg && pending_scale != 0.0)
    hipLaunchKernelGGL((k_correct<T, true, true>), box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, e,
                       chg, n, b, pending_scale);
  else if (chg)
    hipLaunchKernelGGL((k_correct<T, true, false>), box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi,
                       e, chg, n, b, 0.0);
  else
    hipLaunchKernelGGL((k_correct<T, false, false>), box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi,
                       e, nullptr, n, b, 0.0);
  prof_end(st, K_CORRECT, (16.0 + sizeof(T) + (chg ? 8.0 : 0.0)) * box_cells(b));
}
template void launch_correct<float>(double*, const float*, float*, double, int, const Box&,
                                    hipStream_t);
template void launch_correct<double>(double*, const double*, float*, double, int, const Box&,
                                     hipStream_t);

template <typename T, int TXV>
static void correct_est_tiles(double* phi, const T* e, const T* r_old, float* chg,
                              double pending_scale, double kappa, int n, const Box& b,
                              double* partial, const dim3& g, hipStream_t st) {
  const dim3 blk(TXV, 256 / TXV);
  if (chg && pending_scale != 0.0)
    hipLaunchKernelGGL((k_correct_est_v4<T, TXV, true, true>), g, blk, 0, st, phi, e, r_old, chg, n,
                       b, pending_scale, kappa, partial);
  else if (chg)
    hipLaunchKernelGGL((k_correct_est_v4<T, TXV, true, false>), g, blk, 0, st, phi, e, r_old, chg,
                       n, b, 0.0, kappa, partial);
  else
    hipLaunchKernelGGL((k_correct_est_v4<T, TXV, false, false>), g, blk, 0, st, phi, e, r_old,
                       nullptr, n, b, 0.0, kappa, partial);
}

template <typename T>
void launch_correct_est(double* phi, const T* e, const T* r_old, float* chg, double pending_scale,
                        double kappa, int n, const Box& b, double* partial, int* nblocks,
                        hipStream_t st) {
  // the residual's tiles (4 cells per lane; the host asks for this pass only
  // on boxes at least 16 cells wide, where the narrowest tile fits)
  const int ib = b.lo[0] & ~3;
  const int txv = tile_threads(b.hi[0] - ib + 1);
  const unsigned gx = (unsigned)((b.hi[0] - ib + 4 * txv) / (4 * txv));
  const unsigned gy = (unsigned)((b.hi[1] - b.lo[1] + 256 / txv) / (256 / txv));
  const unsigned gz = (unsigned)((b.hi[2] - b.lo[2] + kResKz) / kResKz);
  const dim3 g(gx * gy * gz);
  *nblocks = (int)g.x;
  prof_begin(st, K_CORRECT_EST);
  if (txv == 64)
    correct_est_tiles<T, 64>(phi, e, r_old, chg, pending_scale, kappa, n, b, partial, g, st);
  else if (txv == 32)
    correct_est_tiles<T, 32>(phi, e, r_old, chg, pending_scale, kappa, n, b, partial, g, st);
  else
    correct_est_tiles<T, 16>(phi, e, r_old, chg, pending_scale, kappa, n, b, partial, g, st);
  prof_end(st, K_CORRECT_EST, (16.0 + 2.0 * sizeof(T) + (chg ? 8.0 : 0.0)) * box_cells(b));
}
template void launch_correct_est<float>(double*, const float*, const float*, float*, double,
                                        double, int, const Box&, double*, int*, hipStream_t);
template void launch_correct_est<double>(double*, const double*, const double*, float*, double,
                                         double, int, const Box&, double*, int*, hipStream_t);

void launch_apply_start(double* phi, float* chg, double chg_scale, int n, const Box& b,
                        hipStream_t st) {
  prof_begin(st, K_CORRECT);
  hipLaunchKernelGGL(k_apply_start, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, chg, n, b,
                     chg_scale);
  prof_end(st, K_CORRECT, 24.0 * box_cells(b));
}

// The rhs pass and the first residual of a multigrid solve in one pass (see
// k_rhs_residual_v4) when the box is wide enough for its 4-cell vectors;
// returns false (nothing launched) otherwise.  chg == nullptr: no running
// change; apply: the start d = chg_scale chg is pending afterwards.
template <typename T>
bool launch_rhs_residual(const uint64_t* counts, const double* phi, double* rhs, T* r_out,
                         float* chg, bool apply, double chg_scale, int n, const Box& b,
                         double c_scale, double c_off, double kappa, double* partial,
                         int* nblocks, hipStream_t st, float* g3, double inv2h) {
  const int ib = b.lo[0] & ~3;
  if (b.hi[0] - ib + 1 < 64) return false;
  const int txv = tile_threads(b.hi[0] - ib + 1);
  const unsigned gx = (unsigned)((b.hi[0] - ib + 4 * txv) / (4 * txv));
  const unsigned gy = (unsigned)((b.hi[1] - b.lo[1] + 256 / txv) / (256 / txv));
  const unsigned gz = (unsigned)((b.hi[2] - b.lo[2] + kResKz) / kResKz);
  const int nb = (int)(gx * gy * gz);
  *nblocks = nb;
  const dim3 g(gx * gy * gz), blk(txv, 256 / txv);
  const int mode = chg ? (apply ? 2 : 1) : 0;
  const bool force = g3 != nullptr;
  prof_begin(st, force ? K_RHS_FORCE : K_RHS);
#define SDPM_RR(TX, M, F)                                                                        \
  hipLaunchKernelGGL((k_rhs_residual_v4<T, TX, M, F>), g, blk, 0, st, counts, phi, rhs, r_out,   \
                     chg, n, b, c_scale, c_off, kappa, chg_scale, nb, partial, g3, inv2h)
#define SDPM_RR_TX(M, F)                                                                         \
  if (txv == 64) SDPM_RR(64, M, F); else if (txv == 32) SDPM_RR(32, M, F); else SDPM_RR(16, M, F)
  if (force) {
    if (mode == 2) {
      SDPM_RR_TX(2, true);
    } else if (mode == 1) {
      SDPM_RR_TX(1, true);
    } else {
      SDPM_RR_TX(0, true);
    }
  } else if (mode == 2) {
    SDPM_RR_TX(2, false);
  } else if (mode == 1) {
    SDPM_RR_TX(1, false);
  } else {
    SDPM_RR_TX(0, false);
  }
#undef SDPM_RR_TX
#undef SDPM_RR
  // counts, phi and rhs 8 B each, r sizeof(T); the running change 4 B
  // (read with a start to apply, cleared without); the force mesh 12 B
  prof_end(st, force ? K_RHS_FORCE : K_RHS,
           (24.0 + sizeof(T) + (mode ? 4.0 : 0.0) + (force ? 12.0 : 0.0)) * box_cells(b));
  return true;
}
template bool launch_rhs_residual<float>(const uint64_t*, const double*, double*, float*, float*,
                                         bool, double, int, const Box&, double, double, double,
                                         double*, int*, hipStream_t, float*, double);
template bool launch_rhs_residual<double>(const uint64_t*, const double*, double*, double*, float*,
                                          bool, double, int, const Box&, double, double, double,
                                          double*, int*, hipStream_t, float*, double);

void launch_sum_phi(const double* phi, int n, const Box& b, double* partial, int* nblocks,
                    hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)(g.x * g.y * g.z);
  prof_begin(st, K_SUM_PHI);
  hipLaunchKernelGGL(k_sum_phi, g, dim3(kBoxTx, kBoxTy), 0, st, phi, n, b, partial);
  prof_end(st, K_SUM_PHI, 8.0 * box_cells(b));
}

void launch_add_const(double* phi, float* chg, int n, const Box& b, double v, hipStream_t st) {
  prof_begin(st, K_ADD_CONST);
  hipLaunchKernelGGL(k_add_const, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, chg, n, b, v);
  prof_end(st, K_ADD_CONST, (16.0 + (chg ? 8.0 : 0.0)) * box_cells(b));
}

void launch_reduce_final(const double* partial, int nblocks, int nslots, double* out,
                         hipStream_t st) {
  prof_begin(st, K_REDUCE);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, st, partial, nblocks, nslots, out);
  prof_end(st, K_REDUCE, 8.0 * nblocks * nslots);
}


template <typename T>
void launch_residual_guess(const double* phi, const float* d, double scale, const double* rhs,
                           T* r_out, int n, const Box& b, double kappa, double* partial,
                           int* nblocks, hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)g.x;
  prof_begin(st, K_NET_MISC);
  hipLaunchKernelGGL(k_residual_guess<T>, g, dim3(kBoxTx, kBoxTy), 0, st, phi, d, scale, rhs, r_out,
                     n, b, kappa, partial);
  prof_end(st, K_NET_MISC, (20.0 + sizeof(T)) * box_cells(b));
}
template void launch_residual_guess<float>(const double*, const float*, double, const double*,
                                           float*, int, const Box&, double, double*, int*,
                                           hipStream_t);
template void launch_residual_guess<double>(const double*, const float*, double, const double*,
                                            double*, int, const Box&, double, double*, int*,
                                            hipStream_t);

void launch_apply_guess(double* phi, const float* d, double scale, float* chg, int n,
                        const Box& b, hipStream_t st) {
  prof_begin(st, K_NET_MISC);
  hipLaunchKernelGGL(k_apply_guess, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, d, scale, chg,
                     n, b);
  prof_end(st, K_NET_MISC, (20.0 + (chg ? 8.0 : 0.0)) * box_cells(b));
}


void launch_sum_sq(const double* phi, int n, const Box& b, double* partial, int* nblocks,
                   hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)g.x;
  hipLaunchKernelGGL(k_sum_sq, g, dim3(kBoxTx, kBoxTy), 0, st, phi, n, b, partial);
}

template <typename T>
void launch_record_start(const T* r_split, const double* phi, int n, const Box& b, float* rec,
                         hipStream_t st) {
  const int64_t V = (int64_t)n * n * n;
  hipLaunchKernelGGL(k_record_start<T>, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, r_split,
                     phi, n, b, rec);
}
template void launch_record_start<float>(const float*, const double*, int, const Box&, float*,
                                         hipStream_t);
template void launch_record_start<double>(const double*, const double*, int, const Box&, float*,
                                          hipStream_t);

template <typename T>
void launch_record_accum(const T* e_split, int n, const Box& b, float* dphi, hipStream_t st) {
  hipLaunchKernelGGL(k_record_accum<T>, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, e_split, n, b,
                     dphi);
}
template void launch_record_accum<float>(const float*, int, const Box&, float*, hipStream_t);
template void launch_record_accum<double>(const double*, int, const Box&, float*, hipStream_t);

// Vector width of the colour kernels for a level box (half-row entries);
// 0 (the scalar kernels) for rows under 32 entries.
inline int v4_threads(const Box& b) {
  const int ext = (b.hi[0] >> 1) - ((b.lo[0] >> 1) & ~3) + 1;
  return ext < 32 ? 0 : tile_threads(ext);
}

inline dim3 v4_grid(const Box& b, int txv) {
  const int ty = 256 / txv;
  const int gx = ((b.hi[0] >> 1) - ((b.lo[0] >> 1) & ~3) + 4 * txv) / (4 * txv);
  const int gy = (b.hi[1] - b.lo[1] + ty) / ty;
  const int gz = (b.hi[2] - b.lo[2] + kVecKz) / kVecKz;
  return dim3((unsigned)gx * gy * gz);
}

// One colour sweep; bracket = false leaves its profiling to the caller (a
// group of consecutive sweeps under one event pair).
template <typename T>
static void smooth_color(T* e, const T* r, const Level& L, int level, int color, bool first,
                         T scale, T inv_diag, hipStream_t st, bool bracket = true) {
  const Box& b = L.box;
  const int txv = sizeof(T) == 4 ? v4_threads(b) : 0;   // FP64 levels: the scalar kernel is faster
  if (bracket) prof_begin(st, first ? K_SMOOTH_FIRST : level == 0 ? K_SMOOTH : K_SMOOTH_COARSE);
  const int64_t hc = (int64_t)L.n * L.n * (L.n >> 1);
  T* eo = e + color * hc;
  const T* ex = e + (color ^ 1) * hc;
  const T* ro = r + color * hc;
  if (txv == 64) {
    const dim3 g = v4_grid(b, 64), blk(64, 4);
    if (first)
      hipLaunchKernelGGL((k_smooth_color_v4<T, true, 64>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
    else
      hipLaunchKernelGGL((k_smooth_color_v4<T, false, 64>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
  } else if (txv == 32) {
    const dim3 g = v4_grid(b, 32), blk(32, 8);
    if (first)
      hipLaunchKernelGGL((k_smooth_color_v4<T, true, 32>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
    else
      hipLaunchKernelGGL((k_smooth_color_v4<T, false, 32>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
  } else if (txv == 16) {
    const dim3 g = v4_grid(b, 16), blk(16, 16);
    if (first)
      hipLaunchKernelGGL((k_smooth_color_v4<T, true, 16>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
    else
      hipLaunchKernelGGL((k_smooth_color_v4<T, false, 16>), g, blk, 0, st, eo, ex, ro, L.n, b, color,
                         scale, inv_diag);
  } else {
    const dim3 g = half_grid(b);
    if (first)
      hipLaunchKernelGGL((k_smooth_color<T, true>), g, dim3(kBoxTx, kBoxTy), 0, st, e, r, L.n, b,
                         color, scale, inv_diag);
    else
      hipLaunchKernelGGL((k_smooth_color<T, false>), g, dim3(kBoxTx, kBoxTy), 0, st, e, r, L.n, b,
                         color, scale, inv_diag);
  }
  // first (red, zero guess): r + e of the colour; otherwise e of the other
  // colour + r and e of this colour: half the cells each
  const double cells = (double)box_cells(b);
  if (bracket)
    prof_end(st, first ? K_SMOOTH_FIRST : level == 0 ? K_SMOOTH : K_SMOOTH_COARSE,
             (first ? 1.0 : 1.5) * sizeof(T) * cells);
}

// n consecutive colour sweeps starting with colour c0 (the first with a zero
// guess when zero_first).  On the finest level the non-first sweeps of the
// run share one event bracket: an event pair around each ~140 us sweep left
// the GPU idle ~10 us between two sweeps, ~0.5 ms per 512^3 step.
template <typename T>
static void sweep_run(T* e, const T* r, const Level& L, int level, int c0, int n, bool zero_first,
                      T scale, T inv_diag, hipStream_t st) {
  if (n <= 0) return;
  if (zero_first) {
    smooth_color<T>(e, r, L, level, c0, true, scale, inv_diag, st);
    c0 ^= 1;
    --n;
  }
  const bool group = level == 0 && n > 0;
  if (group) prof_begin(st, K_SMOOTH);
  for (int q = 0; q < n; ++q)
    smooth_color<T>(e, r, L, level, (c0 + q) & 1, false, scale, inv_diag, st, !group);
  if (group) prof_end(st, K_SMOOTH, n * 1.5 * sizeof(T) * (double)box_cells(L.box), n);
}

// Planes per workgroup of the fused sweeps over `cols` columns and nz
// planes: about one workgroup per compute unit (256; each chunk recomputes
// 6 warm-up planes), at least 16 planes (512^3: 128 planes, 0.31 ms against
// 0.33 ms with 64; 256^3: 16 planes, 48 us against 65 us with 32).
static int sweep4_chunk(int cols, int nz) {
  const int per = std::max(1, cols * nz / 256);
  int zc = 16;
  while (zc < nz && zc < per) zc <<= 1;
  return zc;
}

static Box whole_mesh(int n) { return Box{{0, 0, 0}, {n - 1, n - 1, n - 1}}; }

void launch_sweeps4(const float* e, float* e_out, const float* r, int n, float scale, float inv_diag,
                    bool first, bool fused, float* t, float inv_scale, float kappa, const Box* box,
                    hipStream_t st) {
  const Box b = box ? *box : whole_mesh(n);
  if (fused) {
    // 128 x 32-cell columns (one 768-thread workgroup per compute unit: 138
    // KB of LDS, 160 KB with the residual); 64 x 32 on a 64^3 mesh
    // 128-cell columns on periodic levels of 128^3 and up and on boxes in
    // meshes of 512^3 and up; 64-cell columns (two workgroups per CU) on
    // smaller meshes and on the boxes of the 256^3 level, where the chunks
    // of 128-cell columns are short (shrinking phase at 512^3:
    // 11.5 against 11.7 ms per step; on the periodic 256^3 level the wide
    // columns win, 0.72 against 0.86 ms per step)
    const int tx = (n >= 128 && !box) || n >= 512 ? 128 : 64;
    const int ux = tx / 8;
    const int hb = box ? ((b.lo[0] >> 1) & ~3) : 0;
    const int gx = box ? ((b.hi[0] >> 1) - hb + 4 * ux) / (4 * ux) : n / tx;
    const int gy = box ? (b.hi[1] - b.lo[1] + 32) / 32 : n / 32;
    const int nz = b.hi[2] - b.lo[2] + 1;
    const int zc = sweep4_chunk(gx * gy, nz);
    const dim3 g((unsigned)(gx * gy * ((nz + zc - 1) / zc)));
#define SDPM_SWEEP4(F, RS, BX, UXX, NTT)                                                              \
  hipLaunchKernelGGL((k_sweep4<F, RS, BX, UXX, 32, NTT>), g, dim3(NTT), 0, st, e, e_out, r, n, zc,    \
                     scale, inv_diag, t, inv_scale, kappa, b)
#define SDPM_SWEEP4_W(BX, UXX, NTT)               \
  do {                                            \
    if (first && t)                               \
      SDPM_SWEEP4(true, true, BX, UXX, NTT);      \
    else if (first)                               \
      SDPM_SWEEP4(true, false, BX, UXX, NTT);     \
    else if (t)                                   \
      SDPM_SWEEP4(false, true, BX, UXX, NTT);     \
    else                                          \
      SDPM_SWEEP4(false, false, BX, UXX, NTT);    \
  } while (0)
    if (tx == 128) {
      if (box)
        SDPM_SWEEP4_W(true, 16, 768);
      else
        SDPM_SWEEP4_W(false, 16, 768);
    } else {
      if (box)
        SDPM_SWEEP4_W(true, 8, 448);
      else
        SDPM_SWEEP4_W(false, 8, 448);
    }
#undef SDPM_SWEEP4_W
#undef SDPM_SWEEP4
    return;
  }
  if (!first && e != e_out)
    hipMemcpyAsync(e_out, e, (size_t)n * n * n * sizeof(float), hipMemcpyDeviceToDevice, st);
  Level L{};
  L.n = n;
  L.box = b;
  sweep_run<float>(e_out, r, L, 1, 0, 4, first, scale, inv_diag, st);
  if (t) {
    const int txv = v4_threads(b);
    const dim3 g = v4_grid(b, txv);
    if (txv == 64)
      hipLaunchKernelGGL((k_resid_red_v4<float, 64>), g, dim3(64, 4), 0, st, e_out, r, t, n, b,
                         inv_scale, kappa);
    else if (txv == 32)
      hipLaunchKernelGGL((k_resid_red_v4<float, 32>), g, dim3(32, 8), 0, st, e_out, r, t, n, b,
                         inv_scale, kappa);
    else
      hipLaunchKernelGGL((k_resid_red_v4<float, 16>), g, dim3(16, 16), 0, st, e_out, r, t, n, b,
                         inv_scale, kappa);
  }
}

// The fused form of pre or post sweeps on level L when it applies (FP32,
// nsweeps == 2 red-black pairs, a periodic level of at least kSweep4Min
// cells a side with an e_alt array): from a zero guess it writes e, else it
// reads e and writes e_alt, and the two swap.  False when it does not apply.
template <typename T>
static bool sweeps4(Level& L, int level, bool periodic, int nsweeps, bool zero, T scale, T inv_diag,
                    hipStream_t st, bool resid = false, T inv_scale = 0, T kappa = 0) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    const Box fb = whole_mesh(L.n);
    bool whole = true;
    for (int d = 0; d < 3; ++d) whole = whole && L.box.lo[d] == fb.lo[d] && L.box.hi[d] == fb.hi[d];
    // a frozen-exterior box (which keeps a plane from every face) with at
    // least 128^3 cells; periodic levels are whole
    if (nsweeps != 2 || L.n < kSweep4Min || !L.e_alt || (periodic && !whole) ||
        (!periodic && box_cells(L.box) < (int64_t)1 << 21))
      return false;
    // ids: coarser levels; the finest level's passes from the zero guess
    // (with the residual), continuing with the residual (pre-smoothing of a
    // further cycle) and without it (post-smoothing)
    const int id = level > 0 ? K_SWEEP4_COARSE : zero ? K_SWEEP4_FIRST : resid ? K_SWEEP4_RESID : K_SWEEP4;
    prof_begin(st, id);
    float* out = zero ? (float*)L.e : (float*)L.e_alt;
    launch_sweeps4((const float*)L.e, out, (const float*)L.r, L.n, scale, inv_diag, zero, true,
                   resid ? (float*)L.t : nullptr, inv_scale, kappa, periodic ? nullptr : &L.box, st);
    if (!zero) std::swap(L.e, L.e_alt);
    // r read, e written (4 + 4 bytes per cell); without the zero guess the
    // black half of e read too (2 more); with the residual the red half of t
    // written instead of the red half of e (the same 2)
    prof_end(st, id, (zero ? 8.0 : 10.0) * (double)box_cells(L.box));
    return true;
  }
}

template <typename T>
static void resid_red(const T* e, const T* r, T* t, const Level& L, T inv_scale, T kappa,
                      hipStream_t st) {
  const Box& b = L.box;
  const int txv = sizeof(T) == 4 ? v4_threads(b) : 0;
  prof_begin(st, K_RESID_LEVEL);
  if (txv == 64)
    hipLaunchKernelGGL((k_resid_red_v4<T, 64>), v4_grid(b, 64), dim3(64, 4), 0, st, e, r, t, L.n, b,
                       inv_scale, kappa);
  else if (txv == 32)
    hipLaunchKernelGGL((k_resid_red_v4<T, 32>), v4_grid(b, 32), dim3(32, 8), 0, st, e, r, t, L.n, b,
                       inv_scale, kappa);
  else if (txv == 16)
    hipLaunchKernelGGL((k_resid_red_v4<T, 16>), v4_grid(b, 16), dim3(16, 16), 0, st, e, r, t, L.n, b,
                       inv_scale, kappa);
  else
    hipLaunchKernelGGL(k_resid_red<T>, half_grid(b), dim3(kBoxTx, kBoxTy), 0, st, e, r, t, L.n, b,
                       inv_scale, kappa);
  prof_end(st, K_RESID_LEVEL, 2.0 * sizeof(T) * (double)box_cells(b));
}

// r_C = restriction of L's red residual t; the vector form for FP32 levels
// whose fine box takes the vector sweeps.
template <typename T>
static void restrict_level(const Level& L, const Level& C, hipStream_t st) {
  const Box& bc = C.box;
  if constexpr (sizeof(T) == 4) {
    if (v4_threads(L.box)) {
      const int txv = tile_threads(bc.hi[0] - (bc.lo[0] & ~3) + 1);
      const int ty = 256 / txv;
      const unsigned gx = (unsigned)((bc.hi[0] - (bc.lo[0] & ~3) + 4 * txv) / (4 * txv));
      const unsigned gy = (unsigned)((bc.hi[1] - bc.lo[1] + ty) / ty);
      const unsigned gz = (unsigned)((bc.hi[2] - bc.lo[2] + kVecKz) / kVecKz);
      const dim3 g(gx * gy * gz), blk(txv, ty);
      const float* t = (const float*)L.t;
      float* r = (float*)C.r;
      if (txv == 64)
        hipLaunchKernelGGL(k_restrict_v4<64>, g, blk, 0, st, t, r, L.n, C.n, bc);
      else if (txv == 32)
        hipLaunchKernelGGL(k_restrict_v4<32>, g, blk, 0, st, t, r, L.n, C.n, bc);
      else
        hipLaunchKernelGGL(k_restrict_v4<16>, g, blk, 0, st, t, r, L.n, C.n, bc);
      return;
    }
  }
  hipLaunchKernelGGL(k_restrict<T>, box_grid(bc), dim3(kBoxTx, kBoxTy), 0, st, (const T*)L.t,
                     (T*)C.r, L.n, C.n, bc);
}

// e_L += prolongation of e_C on L's black cells (all cells with all_cells);
// the vector form for the black cells of FP32 levels with vector sweeps.
template <typename T>
static void prolong_level(const Level& L, const Level& C, bool all_cells, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    const int txv = v4_threads(L.box);
    if (txv && !all_cells) {
      const dim3 g = v4_grid(L.box, txv), blk(txv, 256 / txv);
      const float* ec = (const float*)C.e;
      float* ef = (float*)L.e;
      if (txv == 64)
        hipLaunchKernelGGL(k_prolong_black_v4<64>, g, blk, 0, st, ec, ef, C.n, L.n, L.box);
      else if (txv == 32)
        hipLaunchKernelGGL(k_prolong_black_v4<32>, g, blk, 0, st, ec, ef, C.n, L.n, L.box);
      else
        hipLaunchKernelGGL(k_prolong_black_v4<16>, g, blk, 0, st, ec, ef, C.n, L.n, L.box);
      return;
    }
  }
  hipLaunchKernelGGL(k_prolong<T>, half_grid(L.box), dim3(kBoxTx, kBoxTy), 0, st, (const T*)C.e,
                     (T*)L.e, C.n, L.n, L.box, all_cells ? 1 : 0);
}

// Red-black sweeps that reduce the slowest mode of level l's operator
// A = Lap_h - 4^l kappa h^2 by 1e-3, red-black Gauss-Seidel taken as the
// square of the Jacobi factor rho = (sum over axes of 2 cos theta_d) /
// (6 + 4^l kappa h^2) of that mode: on a Dirichlet box the lowest sine mode,
// theta_d = pi / (extent_d + 1); on the periodic mesh with kappa > 0 the
// constant mode (theta = 0, rho = 6 / (6 + 4^l kappa h^2)); periodic with
// kappa = 0, where the constant mode is projected out, the lowest nonzero
// mode along one axis, rho = (4 + 2 cos(2 pi / n)) / 6.  A large number
// when rho >= 1.
static int sweeps_for_1e3(const Level& L, int l, double kappa, bool periodic) {
  double num;
  if (periodic) {
    num = kappa > 0.0 ? 6.0 : 4.0 + 2.0 * std::cos(2.0 * M_PI / L.n);
  } else {
    num = 0.0;
    for (int d = 0; d < 3; ++d) num += 2.0 * std::cos(M_PI / (L.box.hi[d] - L.box.lo[d] + 2));
  }
  const double rho = num / (6.0 + std::ldexp(1.0, 2 * l) * kappa);
  if (!(rho > 0.0 && rho < 1.0)) return rho <= 0.0 ? 1 : 1 << 20;
  return std::max(1, (int)std::ceil(std::log(1e-3) / (2.0 * std::log(rho))));
}

template <typename T>
const T* vcycle(Level* lv, int nlev_all, double kappa, int pre, int post, int coarse_sweeps,
                bool periodic, bool fine_start, hipStream_t st) {
  const dim3 blk(kBoxTx, kBoxTy);
  const double es = sizeof(T);
  // The hierarchy ends at the first level below the finest whose own sweeps
  // reach the coarsest solve's 1e-3 in at most pre + post + 1 sweeps: with
  // kappa > 0 the level-l diagonal 6 + 4^l kappa h^2 makes the smoother a
  // fast solver there (kappa h^2 = 0.113 on a 512^3 mesh: factor 0.45 per
  // sweep on the 64^3 level, 5 sweeps), and the levels below it would cost
  // more short launches than the sweeps they replace.  kappa = 0 keeps every
  // level.
  int nlev = nlev_all;
  for (int l = 1; l < nlev_all - 1; ++l)
    if (sweeps_for_1e3(lv[l], l, kappa, periodic) <= pre + post + 1) {
      nlev = l + 1;
      break;
    }
  for (int l = 0; l < nlev - 1; ++l) {
    Level& L = lv[l];
    const double cells = (double)box_cells(L.box);
    const T scale = (T)std::ldexp(1.0, 2 * l);
    const T inv_diag = (T)(1.0 / (6.0 + std::ldexp(1.0, 2 * l) * kappa));
    const T* r = (const T*)L.r;
    // red, black, ... (pre pairs); the first red pass assumes e = 0, except
    // on the finest level when the cycle continues from the correction
    // already there
    const bool zero = !(l == 0 && fine_start);
    const T inv_scale = (T)(1.0 / std::ldexp(1.0, 2 * l));
    // the fused pre-smoothing forms the red residual itself
    if (!sweeps4<T>(L, l, periodic, pre, zero, scale, inv_diag, st, true, inv_scale, (T)kappa)) {
      sweep_run<T>((T*)L.e, r, L, l, 0, 2 * pre, zero, scale, inv_diag, st);
      resid_red<T>((const T*)L.e, r, (T*)L.t, L, inv_scale, (T)kappa, st);
    }
    const Level& C = lv[l + 1];
    prof_begin(st, K_RESTRICT);
    restrict_level<T>(L, C, st);
    prof_end(st, K_RESTRICT, es * (cells / 2 + (double)box_cells(C.box)));
  }
  {
    const int l = nlev - 1;
    const Level& L = lv[l];
    const double sc = std::ldexp(1.0, 2 * l);
    const int nx = L.box.hi[0] - L.box.lo[0] + 1, ny = L.box.hi[1] - L.box.lo[1] + 1,
              nz = L.box.hi[2] - L.box.lo[2] + 1;
    const bool fits = periodic ? (L.n <= kCoarseMax)
                               : ((int64_t)(nx + 2) * (ny + 2) * (nz + 2) <=
                                  (int64_t)kCoarseMax * kCoarseMax * kCoarseMax);
    const T scale = (T)sc, inv_diag = (T)(1.0 / (6.0 + sc * kappa));
    const int sweeps = std::max(1, std::min(coarse_sweeps, sweeps_for_1e3(L, l, kappa, periodic)));
    if (fits) {
      prof_begin(st, K_COARSE);
      hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(1024), 0, st, (T*)L.e, (const T*)L.r, L.n,
                         L.box, scale, inv_diag, sweeps,
                         (periodic && kappa == 0.0) ? 1 : 0, periodic ? 1 : 0);
      prof_end(st, K_COARSE, 2 * es * (double)box_cells(L.box));
    } else {
      // a coarsest level beyond the LDS solve (a large degenerate Dirichlet
      // box, or a level the hierarchy ends on early): sweeps through global
      // memory
      for (int s = 0; s < sweeps; ++s) {
        smooth_color<T>((T*)L.e, (const T*)L.r, L, l, 0, s == 0, scale, inv_diag, st);
        smooth_color<T>((T*)L.e, (const T*)L.r, L, l, 1, false, scale, inv_diag, st);
      }
    }
  }
  for (int l = nlev - 2; l >= 0; --l) {
    Level& L = lv[l];
    const Level& C = lv[l + 1];
    const double cells = (double)box_cells(L.box);
    const T scale = (T)std::ldexp(1.0, 2 * l);
    const T inv_diag = (T)(1.0 / (6.0 + std::ldexp(1.0, 2 * l) * kappa));
    prof_begin(st, K_PROLONG);
    prolong_level<T>(L, C, post == 0, st);
    prof_end(st, K_PROLONG, es * ((post > 0 ? 1.0 : 2.0) * cells + (double)box_cells(C.box)));
    if (!sweeps4<T>(L, l, periodic, post, false, scale, inv_diag, st))
      sweep_run<T>((T*)L.e, (const T*)L.r, L, l, 0, 2 * post, false, scale, inv_diag, st);
  }
  return (const T*)lv[0].e;
}
template const float* vcycle<float>(Level*, int, double, int, int, int, bool, bool, hipStream_t);
template const double* vcycle<double>(Level*, int, double, int, int, int, bool, bool, hipStream_t);

}  // namespace sdpm
