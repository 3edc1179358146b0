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

__device__ inline int block_linear() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ a, int n, Box b, T v) {
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) a[lin(i, j, k, n)] = v;
}

// ----------------------------------------------------------- FP64 kernels
// rhs = C * c_scale - c_off - kappa phi ; partial sum of rhs^2.
__global__ void __launch_bounds__(256)
k_rhs(const uint64_t* __restrict__ counts, const double* __restrict__ phi,
      double* __restrict__ rhs, int n, Box b, double c_scale, double c_off, double kappa,
      double* __restrict__ partial) {
  __shared__ double sh[4];
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    for (int k = k0; k <= k1; ++k) {
      const int64_t c = lin(i, j, k, n);
      const double v = (double)counts[c] * c_scale - c_off - kappa * phi[c];
      rhs[c] = v;
      acc += v * v;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

// r = rhs - (Lap_h phi - kappa phi) in FP64, stored as T; partial sum of r^2.
template <typename T>
__global__ void __launch_bounds__(256)
k_residual(const double* __restrict__ phi, const double* __restrict__ rhs,
           T* __restrict__ rout, int n, Box b, double kappa, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  const int m = n - 1;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    const int ip = (i + 1) & m, im = (i - 1) & m, jp = (j + 1) & m, jm = (j - 1) & m;
    for (int k = k0; k <= k1; ++k) {
      const int kp = (k + 1) & m, km = (k - 1) & m;
      const int64_t c = lin(i, j, k, n);
      const double ctr = phi[c];
      const double nb = phi[lin(ip, j, k, n)] + phi[lin(im, j, k, n)] + phi[lin(i, jp, k, n)] +
                        phi[lin(i, jm, k, n)] + phi[lin(i, j, kp, n)] + phi[lin(i, j, km, n)];
      const double res = rhs[c] - (nb - 6.0 * ctr - kappa * ctr);
      rout[c] = (T)res;
      acc += res * res;
    }
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_correct(double* __restrict__ phi, const T* __restrict__ e, int n, Box b) {
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    phi[c] += (double)e[c];
  }
}

__global__ void __launch_bounds__(256)
k_sum_phi(const double* __restrict__ phi, int n, Box b, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  double acc = 0.0;
  if (i <= b.hi[0] && j <= b.hi[1]) {
    const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
    const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
    for (int k = k0; k <= k1; ++k) acc += phi[lin(i, j, k, n)];
  }
  const double s = block_sum<256>(acc, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[block_linear()] = s;
}

__global__ void __launch_bounds__(256) k_add_const(double* __restrict__ phi, int n, Box b, double v) {
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) phi[lin(i, j, k, n)] += v;
}

// out[s] = sum of partial[s * nblocks + 0 .. nblocks), fixed order.
__global__ void __launch_bounds__(1024)
k_reduce_final(const double* __restrict__ partial, int nblocks, int nslots,
               double* __restrict__ out) {
  __shared__ double sh[16];
  for (int s = 0; s < nslots; ++s) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < nblocks; t += 1024) acc += partial[(int64_t)s * nblocks + t];
    const double r = block_sum<1024>(acc, sh);
    if (threadIdx.x == 0) out[s] = r;
  }
}

// -------------------------------------------------------- multigrid (T)
// Zero initial guess: one red half-sweep is e = -4^l r / diag on red cells,
// and black cells start at 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_smooth_first(T* __restrict__ e, const T* __restrict__ r, int n, Box b, T scale, T inv_diag) {
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  for (int k = k0; k <= k1; ++k) {
    const int64_t c = lin(i, j, k, n);
    e[c] = ((i + j + k) & 1) == 0 ? -scale * r[c] * inv_diag : (T)0;
  }
}

// One colour of red-black Gauss-Seidel: cells with (i+j+k)&1 == color.
// A workgroup row of 64 threads covers 128 cells in x.
template <typename T>
__global__ void __launch_bounds__(256)
k_smooth(T* __restrict__ e, const T* __restrict__ r, int n, Box b, int color, T scale,
         T inv_diag) {
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (j > b.hi[1]) return;
  const int t = blockIdx.x * kBoxTx + threadIdx.x;
  const int m = n - 1;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int jp = (j + 1) & m, jm = (j - 1) & m;
  for (int k = k0; k <= k1; ++k) {
    const int par = (b.lo[0] + j + k) & 1;
    const int i = b.lo[0] + (par ^ color) + 2 * t;
    if (i > b.hi[0]) continue;
    const int kp = (k + 1) & m, km = (k - 1) & m;
    const int64_t c = lin(i, j, k, n);
    const T nb = e[lin((i + 1) & m, j, k, n)] + e[lin((i - 1) & m, j, k, n)] + e[lin(i, jp, k, n)] +
                 e[lin(i, jm, k, n)] + e[lin(i, j, kp, n)] + e[lin(i, j, km, n)];
    e[c] = (nb - scale * r[c]) * inv_diag;
  }
}

// t = r - A_l e on the box.
template <typename T>
__global__ void __launch_bounds__(256)
k_resid_level(const T* __restrict__ e, const T* __restrict__ r, T* __restrict__ tout, int n,
              Box b, T inv_scale, T kappa) {
  const int i = b.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = b.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > b.hi[0] || j > b.hi[1]) return;
  const int m = n - 1;
  const int k0 = b.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, b.hi[2]);
  const int ip = (i + 1) & m, im = (i - 1) & m, jp = (j + 1) & m, jm = (j - 1) & m;
  for (int k = k0; k <= k1; ++k) {
    const int kp = (k + 1) & m, km = (k - 1) & m;
    const int64_t c = lin(i, j, k, n);
    const T ctr = e[c];
    const T nb = e[lin(ip, j, k, n)] + e[lin(im, j, k, n)] + e[lin(i, jp, k, n)] +
                 e[lin(i, jm, k, n)] + e[lin(i, j, kp, n)] + e[lin(i, j, km, n)];
    tout[c] = r[c] - (nb - (T)6 * ctr) * inv_scale + kappa * ctr;
  }
}

// Full weighting: r_c(I) = sum_{o in {-1,0,1}^3} w(o) t_f(2I + o),
// w = (1/4, 1/2, 1/4) per axis.  t_f is zero outside the fine box.
template <typename T>
__global__ void __launch_bounds__(256)
k_restrict(const T* __restrict__ tf, T* __restrict__ rc, int nf, int nc, Box bc) {
  const int I = bc.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int J = bc.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (I > bc.hi[0] || J > bc.hi[1]) return;
  const int m = nf - 1;
  const int K0 = bc.lo[2] + blockIdx.z * kBoxKz;
  const int K1 = min(K0 + kBoxKz - 1, bc.hi[2]);
  const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
  for (int K = K0; K <= K1; ++K) {
    T acc = 0;
    for (int oz = -1; oz <= 1; ++oz) {
      const int kf = (2 * K + oz) & m;
      T az = 0;
      for (int oy = -1; oy <= 1; ++oy) {
        const int jf = (2 * J + oy) & m;
        const int64_t row = lin(0, jf, kf, nf);
        const T ax = w[0] * tf[row + ((2 * I - 1) & m)] + w[1] * tf[row + 2 * I] +
                     w[2] * tf[row + ((2 * I + 1) & m)];
        az += w[oy + 1] * ax;
      }
      acc += w[oz + 1] * az;
    }
    rc[lin(I, J, K, nc)] = acc;
  }
}

// Trilinear prolongation and correction: e_f += P e_c on the fine box.
// Coarse values outside the coarse box are zero.
template <typename T>
__global__ void __launch_bounds__(256)
k_prolong(const T* __restrict__ ec, T* __restrict__ ef, int nc, int nf, Box bf) {
  const int i = bf.lo[0] + blockIdx.x * kBoxTx + threadIdx.x;
  const int j = bf.lo[1] + blockIdx.y * kBoxTy + threadIdx.y;
  if (i > bf.hi[0] || j > bf.hi[1]) return;
  const int mc = nc - 1;
  const int k0 = bf.lo[2] + blockIdx.z * kBoxKz;
  const int k1 = min(k0 + kBoxKz - 1, bf.hi[2]);
  const int i0 = i >> 1, i1 = ((i >> 1) + (i & 1)) & mc;
  const int j0 = j >> 1, j1 = ((j >> 1) + (j & 1)) & mc;
  const T wi = (i & 1) ? (T)0.5 : (T)1, wj = (j & 1) ? (T)0.5 : (T)1;
  for (int k = k0; k <= k1; ++k) {
    const int k0c = k >> 1, k1c = ((k >> 1) + (k & 1)) & mc;
    const T wk = (k & 1) ? (T)0.5 : (T)1;
    T v;
    if (!(i & 1) && !(j & 1) && !(k & 1)) {
      v = ec[lin(i0, j0, k0c, nc)];
    } else {
      // an odd index averages its two coarse neighbours (weight 1/2 each),
      // an even index takes its coincident coarse value (weight 1)
      v = 0;
      const int is[2] = {i0, i1}, js[2] = {j0, j1}, ks[2] = {k0c, k1c};
      const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
      for (int c = 0; c < nk; ++c)
        for (int bb = 0; bb < nj; ++bb)
          for (int a = 0; a < ni; ++a) v += ec[lin(is[a], js[bb], ks[c], nc)];
      v *= wi * wj * wk;
    }
    ef[lin(i, j, k, nf)] += v;
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
    gidx[u] = lin(i, j, k, n);
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

}  // namespace

// ------------------------------------------------------------- launchers
template <typename T>
void launch_fill(T* a, int n, const Box& b, T v, hipStream_t st) {
  prof_begin(st);
  hipLaunchKernelGGL(k_fill<T>, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, a, n, b, v);
  prof_end(st, K_FILL, (double)box_cells(b) * sizeof(T));
}
template void launch_fill<float>(float*, int, const Box&, float, hipStream_t);
template void launch_fill<double>(double*, int, const Box&, double, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, int, const Box&, uint64_t, hipStream_t);

void launch_rhs(const uint64_t* counts, const double* phi, double* rhs, int n, const Box& b,
                double c_scale, double c_off, double kappa, double* partial, int* nblocks,
                hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)(g.x * g.y * g.z);
  prof_begin(st);
  hipLaunchKernelGGL(k_rhs, g, dim3(kBoxTx, kBoxTy), 0, st, counts, phi, rhs, n, b, c_scale,
                     c_off, kappa, partial);
  prof_end(st, K_RHS, 24.0 * box_cells(b));
}

template <typename T>
void launch_residual(const double* phi, const double* rhs, T* r_out, int n, const Box& b,
                     double kappa, double* partial, int* nblocks, hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)(g.x * g.y * g.z);
  prof_begin(st);
  hipLaunchKernelGGL(k_residual<T>, g, dim3(kBoxTx, kBoxTy), 0, st, phi, rhs, r_out, n, b,
                     kappa, partial);
  prof_end(st, K_RESIDUAL, (16.0 + sizeof(T)) * box_cells(b));
}
template void launch_residual<float>(const double*, const double*, float*, int, const Box&,
                                     double, double*, int*, hipStream_t);
template void launch_residual<double>(const double*, const double*, double*, int, const Box&,
                                      double, double*, int*, hipStream_t);

template <typename T>
void launch_correct(double* phi, const T* e, int n, const Box& b, hipStream_t st) {
  prof_begin(st);
  hipLaunchKernelGGL(k_correct<T>, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, e, n, b);
  prof_end(st, K_CORRECT, (16.0 + sizeof(T)) * box_cells(b));
}
template void launch_correct<float>(double*, const float*, int, const Box&, hipStream_t);
template void launch_correct<double>(double*, const double*, int, const Box&, hipStream_t);

void launch_sum_phi(const double* phi, int n, const Box& b, double* partial, int* nblocks,
                    hipStream_t st) {
  const dim3 g = box_grid(b);
  *nblocks = (int)(g.x * g.y * g.z);
  prof_begin(st);
  hipLaunchKernelGGL(k_sum_phi, g, dim3(kBoxTx, kBoxTy), 0, st, phi, n, b, partial);
  prof_end(st, K_SUM_PHI, 8.0 * box_cells(b));
}

void launch_add_const(double* phi, int n, const Box& b, double v, hipStream_t st) {
  prof_begin(st);
  hipLaunchKernelGGL(k_add_const, box_grid(b), dim3(kBoxTx, kBoxTy), 0, st, phi, n, b, v);
  prof_end(st, K_ADD_CONST, 16.0 * box_cells(b));
}

void launch_reduce_final(const double* partial, int nblocks, int nslots, double* out,
                         hipStream_t st) {
  prof_begin(st);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, st, partial, nblocks, nslots, out);
  prof_end(st, K_REDUCE, 8.0 * nblocks * nslots);
}

template <typename T>
void vcycle(const Level* lv, int nlev, double kappa, int pre, int post, int coarse_sweeps,
            bool periodic, hipStream_t st) {
  const dim3 blk(kBoxTx, kBoxTy);
  const double es = sizeof(T);
  for (int l = 0; l < nlev - 1; ++l) {
    const Level& L = lv[l];
    const double cells = (double)box_cells(L.box);
    const T scale = (T)std::ldexp(1.0, 2 * l);
    const T inv_diag = (T)(1.0 / (6.0 + std::ldexp(1.0, 2 * l) * kappa));
    const dim3 g = box_grid(L.box), gc = box_grid(L.box, 2 * kBoxTx);
    T* e = (T*)L.e;
    const T* r = (const T*)L.r;
    for (int s = 0; s < pre; ++s) {
      prof_begin(st);
      if (s == 0) {
        hipLaunchKernelGGL(k_smooth_first<T>, g, blk, 0, st, e, r, L.n, L.box, scale, inv_diag);
        prof_end(st, K_SMOOTH_FIRST, 2 * es * cells);
      } else {
        hipLaunchKernelGGL(k_smooth<T>, gc, blk, 0, st, e, r, L.n, L.box, 0, scale, inv_diag);
        prof_end(st, K_SMOOTH, 2 * es * cells);
      }
      prof_begin(st);
      hipLaunchKernelGGL(k_smooth<T>, gc, blk, 0, st, e, r, L.n, L.box, 1, scale, inv_diag);
      prof_end(st, K_SMOOTH, 2 * es * cells);
    }
    prof_begin(st);
    hipLaunchKernelGGL(k_resid_level<T>, g, blk, 0, st, e, r, (T*)L.t, L.n, L.box,
                       (T)(1.0 / std::ldexp(1.0, 2 * l)), (T)kappa);
    prof_end(st, K_RESID_LEVEL, 3 * es * cells);
    const Level& C = lv[l + 1];
    prof_begin(st);
    hipLaunchKernelGGL(k_restrict<T>, box_grid(C.box), blk, 0, st, (const T*)L.t, (T*)C.r, L.n,
                       C.n, C.box);
    prof_end(st, K_RESTRICT, es * (cells + (double)box_cells(C.box)));
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
    // sweeps for a 1e-3 reduction of the slowest mode: Jacobi factor
    // rho = 6 cos(theta) / (6 + 4^l kappa h^2), red-black GS factor rho^2,
    // theta = 2 pi / n (periodic) or pi / (extent + 1) (Dirichlet)
    int sweeps = coarse_sweeps;
    {
      const int ext = std::max(nx, std::max(ny, nz));
      const double th = periodic ? 2.0 * M_PI / L.n : M_PI / (ext + 1);
      const double rho = 6.0 * std::cos(th) / (6.0 + sc * kappa);
      if (rho > 0.0 && rho < 1.0) {
        const int need = (int)std::ceil(std::log(1e-3) / (2.0 * std::log(rho)));
        sweeps = std::max(1, std::min(coarse_sweeps, need));
      }
    }
    if (fits) {
      prof_begin(st);
      hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(1024), 0, st, (T*)L.e, (const T*)L.r, L.n,
                         L.box, scale, inv_diag, sweeps,
                         (periodic && kappa == 0.0) ? 1 : 0, periodic ? 1 : 0);
      prof_end(st, K_COARSE, 2 * es * (double)box_cells(L.box));
    } else {
      // large degenerate Dirichlet box: sweeps through global memory
      const dim3 g = box_grid(L.box), gc = box_grid(L.box, 2 * kBoxTx);
      const double cells = (double)box_cells(L.box);
      prof_begin(st);
      hipLaunchKernelGGL(k_smooth_first<T>, g, blk, 0, st, (T*)L.e, (const T*)L.r, L.n, L.box,
                         scale, inv_diag);
      prof_end(st, K_SMOOTH_FIRST, 2 * es * cells);
      for (int s = 0; s < 2 * sweeps - 1; ++s) {
        prof_begin(st);
        hipLaunchKernelGGL(k_smooth<T>, gc, blk, 0, st, (T*)L.e, (const T*)L.r, L.n, L.box,
                           (s + 1) & 1, scale, inv_diag);
        prof_end(st, K_SMOOTH, 2 * es * cells);
      }
    }
  }
  for (int l = nlev - 2; l >= 0; --l) {
    const Level& L = lv[l];
    const Level& C = lv[l + 1];
    const double cells = (double)box_cells(L.box);
    const T scale = (T)std::ldexp(1.0, 2 * l);
    const T inv_diag = (T)(1.0 / (6.0 + std::ldexp(1.0, 2 * l) * kappa));
    prof_begin(st);
    hipLaunchKernelGGL(k_prolong<T>, box_grid(L.box), blk, 0, st, (const T*)C.e, (T*)L.e, C.n,
                       L.n, L.box);
    prof_end(st, K_PROLONG, es * (2 * cells + (double)box_cells(C.box)));
    const dim3 gc = box_grid(L.box, 2 * kBoxTx);
    for (int s = 0; s < post; ++s) {
      for (int color = 0; color < 2; ++color) {
        prof_begin(st);
        hipLaunchKernelGGL(k_smooth<T>, gc, blk, 0, st, (T*)L.e, (const T*)L.r, L.n, L.box, color,
                           scale, inv_diag);
        prof_end(st, K_SMOOTH, 2 * es * cells);
      }
    }
  }
}
template void vcycle<float>(const Level*, int, double, int, int, int, bool, hipStream_t);
template void vcycle<double>(const Level*, int, double, int, int, int, bool, hipStream_t);

}  // namespace sdpm
