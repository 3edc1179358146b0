// Power spectrum of particle positions in a periodic box: the accuracy metric
// the paper compares runs with (Sec. 3.1, Sec. 3.2: 3D spectra of the
// lightcone in a cubical box of the original size), with the discreteness
// corrections of Jing (2005) that the paper names for its spectrum tool
// (Sec. 2.4).
//
// delta = C / (nbar 2^(3B)) - 1 from the fixed-point CIC deposit (the step's
// own deposit kernel, no drift), one FP64 real-to-complex FFT, then shell
// sums over the half spectrum: a column 0 < i < n/2 stands for itself and
// its conjugate mode, the columns i = 0 and i = n/2 for themselves.  Shell
// b = rint(|f|) in 1 .. n/2, f the signed integer frequency (index n/2 is
// -n/2).  Per shell: mean |k|, modes, mean L^3 |delta_k|^2, mean of the CIC
// shot-noise alias factor C1(f) = prod_d (1 - 2/3 sin^2(pi f_d / n)); Jing's
// correction divides the shot-subtracted mean by the shell mean of
//   S(f) = sum_{m in [-2,2]^3} W^2(f + n m) (|f + n m| / |f|)^neff,
// W^2(g) = prod_d sinc^4(pi g_d / n), the local slope neff re-estimated
// three times from the corrected spectrum (central log-log differences of
// neighbouring shells, one-sided at the ends, clamped to [-4, 4], 0 where a
// neighbour is not positive).  Where a frequency equals -n/2 the conjugate
// mode's frequencies are not -f (index n/2 maps to -n/2 both ways), so its S
// is evaluated on its own.  Shell sums are accumulated per workgroup in LDS
// and reduced over a fixed number of workgroups in a fixed order.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace sdpm {
namespace {

constexpr int kPkBlocks = 1024;     // workgroups of the shell passes
constexpr int kPkImages = 2;        // images per axis side in S
constexpr int kPkTab = 2 * kPkImages + 1;
constexpr int kPkIter = 3;
constexpr int kPkSums = 4;          // P_raw, C1, |f|, weight (S pass: S)

__device__ inline int freq(int idx, int n) { return idx < n / 2 ? idx : idx - n; }

__global__ void __launch_bounds__(256)
k_pk_delta(double* __restrict__ mesh, int64_t cells, double inv) {
  // counts (u64) -> delta (double) in place
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cells;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = ((const uint64_t*)mesh)[q];
    mesh[q] = (double)c * inv - 1.0;
  }
}

// tab[(f + n/2) * kPkTab + m + kPkImages] = sinc^4(pi (f + n m) / n),
// sq[(f + n/2) * kPkTab + ...] = (f + n m)^2
__device__ inline double s_of(int fx, int fy, int fz, int n, double neff, const double* tab,
                              const double* sq) {
  const double f2 = (double)fx * fx + (double)fy * fy + (double)fz * fz;
  const int ox = (fx + n / 2) * kPkTab, oy = (fy + n / 2) * kPkTab, oz = (fz + n / 2) * kPkTab;
  double s = 0.0;
  for (int a = 0; a < kPkTab; ++a) {
    const double wx = tab[ox + a], gx = sq[ox + a];
    for (int b = 0; b < kPkTab; ++b) {
      const double wxy = wx * tab[oy + b], gxy = gx + sq[oy + b];
      for (int c = 0; c < kPkTab; ++c) {
        const double w = wxy * tab[oz + c];
        if (neff == 0.0) {
          s += w;
        } else {
          const double r = (gxy + sq[oz + c]) / f2;
          s += w * exp(0.5 * neff * log(r));
        }
      }
    }
  }
  return s;
}

// RAW: per shell sums of w P_raw, w C1, w |f|, w; else: w S(f; neff[shell])
template <bool RAW>
__global__ void __launch_bounds__(256)
k_pk_shells(const hipfftDoubleComplex* __restrict__ c, int n, double l3, const double* neff,
            const double* tab, const double* sq, double* __restrict__ partial) {
  extern __shared__ double acc[];
  const int nb = n / 2;
  const int nsum = RAW ? kPkSums : 1;
  for (int q = threadIdx.x; q < nb * nsum; q += blockDim.x) acc[q] = 0.0;
  __syncthreads();
  const int hx = n / 2 + 1;
  const int64_t total = (int64_t)n * n * hx;
  const double inv_n3 = 1.0 / ((double)n * n * n);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % hx);
    const int64_t r = q / hx;
    const int j = (int)(r % n), k = (int)(r / n);
    const int fx = i == n / 2 ? -n / 2 : i, fy = freq(j, n), fz = freq(k, n);
    const double fa = sqrt((double)fx * fx + (double)fy * fy + (double)fz * fz);
    const int shell = (int)rint(fa);
    if (shell < 1 || shell > nb) continue;
    const bool pair = i > 0 && i < n / 2;
    const double w = pair ? 2.0 : 1.0;
    const int sb = shell - 1;
    if (RAW) {
      const hipfftDoubleComplex v = c[q];
      const double re = v.x * inv_n3, im = v.y * inv_n3;
      double c1 = 1.0;
      const int fs[3] = {fx, fy, fz};
      for (int d = 0; d < 3; ++d) {
        const double s = sin(M_PI * fs[d] / n);
        c1 *= 1.0 - (2.0 / 3.0) * s * s;
      }
      atomicAdd(&acc[sb * kPkSums + 0], w * l3 * (re * re + im * im));
      atomicAdd(&acc[sb * kPkSums + 1], w * c1);
      atomicAdd(&acc[sb * kPkSums + 2], w * fa);
      atomicAdd(&acc[sb * kPkSums + 3], w);
    } else {
      const double ne = neff[sb];
      double s = s_of(fx, fy, fz, n, ne, tab, sq);
      if (pair) {
        // the conjugate mode: frequencies of index (n - i, -j mod n, -k mod n)
        const int px = -fx, py = freq((n - j) % n, n), pz = freq((n - k) % n, n);
        s += (py == -fy && pz == -fz) ? s : s_of(px, py, pz, n, ne, tab, sq);
      }
      atomicAdd(&acc[sb], s);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nb * nsum; q += blockDim.x)
    partial[(int64_t)blockIdx.x * nb * nsum + q] = acc[q];
}

// out[q] = sum over workgroups of partial[b][q], fixed order
__global__ void __launch_bounds__(256)
k_pk_reduce(const double* __restrict__ partial, int nblocks, int width, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= width) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * width + q];
  out[q] = s;
}

struct PkLayout {
  size_t mesh, cbuf, work, tab, sq, partial, sums, neff, flags, total;
};

PkLayout pk_layout(int n) {
  PkLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  const int nb = n / 2;
  l.mesh = take((size_t)n * n * n * sizeof(double));
  l.cbuf = take(fft_complex_bytes(n));
  l.work = take(fft_complex_bytes(n));
  l.tab = take((size_t)(n + 1) * kPkTab * sizeof(double));
  l.sq = take((size_t)(n + 1) * kPkTab * sizeof(double));
  l.partial = take((size_t)kPkBlocks * nb * kPkSums * sizeof(double));
  l.sums = take((size_t)nb * kPkSums * sizeof(double));
  l.neff = take((size_t)nb * sizeof(double));
  l.flags = take(16 * sizeof(uint32_t));
  l.total = off;
  return l;
}

void slopes(const std::vector<double>& k, const std::vector<double>& p, std::vector<double>* out) {
  const int nb = (int)k.size();
  for (int b = 0; b < nb; ++b) {
    const int lo = std::max(b - 1, 0), hi = std::min(b + 1, nb - 1);
    double v = 0.0;
    if (hi != lo && p[lo] > 0.0 && p[hi] > 0.0 && k[lo] > 0.0)
      v = std::min(std::max(std::log(p[hi] / p[lo]) / std::log(k[hi] / k[lo]), -4.0), 4.0);
    (*out)[b] = v;
  }
}

}  // namespace

size_t pk_workspace_bytes(int n) { return pk_layout(n).total; }

int power_spectrum(const double* const x[3], int64_t npart, double box, int n, int flags,
                   void* ws, hipStream_t st, double* k_out, double* p_out, double* praw_out,
                   int64_t* modes_out, char* msg, size_t len) {
  const PkLayout lay = pk_layout(n);
  char* base = (char*)ws;
  double* mesh = (double*)(base + lay.mesh);
  auto* cbuf = (hipfftDoubleComplex*)(base + lay.cbuf);
  double* tab = (double*)(base + lay.tab);
  double* sq = (double*)(base + lay.sq);
  double* partial = (double*)(base + lay.partial);
  double* sums = (double*)(base + lay.sums);
  double* neff_dev = (double*)(base + lay.neff);
  uint32_t* dflags = (uint32_t*)(base + lay.flags);
  const int nb = n / 2;
  const int frac_bits = 14;
  auto herr = [&](const char* what) {
    snprintf(msg, len, "%s", what);
    return SDPM_EHIP;
  };
  // CIC counts of the positions (periodic box, no drift)
  if (hipMemsetAsync(dflags, 0, 16 * sizeof(uint32_t), st) != hipSuccess) return herr("memset");
  Box full;
  for (int d = 0; d < 3; ++d) full.lo[d] = 0, full.hi[d] = n - 1;
  launch_fill<uint64_t>((uint64_t*)mesh, n, full, 0ull, st);
  ParticleArgs pa{};
  for (int d = 0; d < 3; ++d) pa.x[d] = const_cast<double*>(x[d]), pa.p[d] = nullptr;
  pa.id = nullptr;
  pa.n = npart;
  MeshMap mm{};
  mm.ng = n;
  mm.frac_bits = frac_bits;
  mm.periodic = 1;
  mm.box = box;
  mm.scale = (double)n * std::ldexp(1.0, frac_bits) / box;
  mm.active = full;
  launch_drift_deposit<double>(pa, 0.0, 0, mm, (uint64_t*)mesh, dflags, st);
  uint32_t hflags = 0;
  if (hipMemcpyAsync(&hflags, dflags, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return herr("deposit failed");
  if (hflags) {
    snprintf(msg, len, "a position lies outside [0, box] or is not finite");
    return SDPM_EDOMAIN;
  }
  const int64_t cells = (int64_t)n * n * n;
  const double nbar = (double)npart / (double)cells;
  hipLaunchKernelGGL(k_pk_delta, dim3(4096), dim3(256), 0, st, mesh, cells,
                     1.0 / (nbar * std::ldexp(1.0, 3 * frac_bits)));
  // FFT
  hipfftHandle plan = nullptr;
  size_t wneed = 0;
  if (hipfftCreate(&plan) != HIPFFT_SUCCESS) return herr("hipfftCreate failed");
  bool ok = hipfftSetAutoAllocation(plan, 0) == HIPFFT_SUCCESS &&
            hipfftMakePlan3d(plan, n, n, n, HIPFFT_D2Z, &wneed) == HIPFFT_SUCCESS &&
            wneed <= fft_complex_bytes(n) &&
            hipfftSetWorkArea(plan, base + lay.work) == HIPFFT_SUCCESS &&
            hipfftSetStream(plan, st) == HIPFFT_SUCCESS &&
            hipfftExecD2Z(plan, (hipfftDoubleReal*)mesh, cbuf) == HIPFFT_SUCCESS;
  if (!ok) {
    hipfftDestroy(plan);
    return herr("hipFFT plan or execution failed");
  }
  // window tables
  std::vector<double> htab((size_t)(n + 1) * kPkTab), hsq((size_t)(n + 1) * kPkTab);
  for (int f = -n / 2; f <= n / 2; ++f)
    for (int m = -kPkImages; m <= kPkImages; ++m) {
      const double g = (double)f + (double)n * m;
      const double xg = M_PI * g / n;
      const double sc = g == 0.0 ? 1.0 : std::sin(xg) / xg;
      htab[(size_t)(f + n / 2) * kPkTab + m + kPkImages] = sc * sc * sc * sc;
      hsq[(size_t)(f + n / 2) * kPkTab + m + kPkImages] = g * g;
    }
  if (hipMemcpyAsync(tab, htab.data(), htab.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(sq, hsq.data(), hsq.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
          hipSuccess) {
    hipfftDestroy(plan);
    return herr("copy of the window tables failed");
  }
  // shell sums of the raw spectrum
  const double l3 = box * box * box;
  std::vector<double> raw((size_t)nb * kPkSums);
  prof_begin(st, K_PK);
  hipLaunchKernelGGL(k_pk_shells<true>, dim3(kPkBlocks), dim3(256),
                     (size_t)nb * kPkSums * sizeof(double), st, cbuf, n, l3, neff_dev, tab, sq,
                     partial);
  prof_end(st, K_PK, 16.0 * (double)n * n * (n / 2 + 1));
  hipLaunchKernelGGL(k_pk_reduce, dim3((nb * kPkSums + 255) / 256), dim3(256), 0, st, partial,
                     kPkBlocks, nb * kPkSums, sums);
  ok = hipMemcpyAsync(raw.data(), sums, raw.size() * sizeof(double), hipMemcpyDeviceToHost, st) ==
           hipSuccess &&
       hipStreamSynchronize(st) == hipSuccess;
  hipfftDestroy(plan);
  if (!ok) return herr("shell sums failed");
  const double kf = 2.0 * M_PI / box;
  std::vector<double> kmean(nb), praw(nb), c1(nb), signal(nb), p(nb), neff(nb, 0.0), ssum(nb);
  const double shot = (flags & SDPM_PK_SHOT) ? l3 / (double)npart : 0.0;
  for (int b = 0; b < nb; ++b) {
    const double wsum = raw[b * kPkSums + 3];
    modes_out[b] = (int64_t)llround(wsum);
    const double inv = wsum > 0.0 ? 1.0 / wsum : 0.0;
    praw[b] = raw[b * kPkSums + 0] * inv;
    c1[b] = raw[b * kPkSums + 1] * inv;
    kmean[b] = raw[b * kPkSums + 2] * inv * kf;
    signal[b] = praw[b] - shot * c1[b];
    p[b] = signal[b];
  }
  if (flags & SDPM_PK_JING) {
    for (int it = 0; it <= kPkIter; ++it) {
      if (hipMemcpyAsync(neff_dev, neff.data(), nb * sizeof(double), hipMemcpyHostToDevice, st) !=
          hipSuccess)
        return herr("copy of the slopes failed");
      prof_begin(st, K_PK);
      hipLaunchKernelGGL(k_pk_shells<false>, dim3(kPkBlocks), dim3(256), (size_t)nb * sizeof(double),
                         st, cbuf, n, l3, neff_dev, tab, sq, partial);
      prof_end(st, K_PK, 0.0);
      hipLaunchKernelGGL(k_pk_reduce, dim3((nb + 255) / 256), dim3(256), 0, st, partial, kPkBlocks,
                         nb, sums);
      if (hipMemcpyAsync(ssum.data(), sums, nb * sizeof(double), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return herr("alias sums failed");
      for (int b = 0; b < nb; ++b) {
        const double wsum = raw[b * kPkSums + 3];
        p[b] = ssum[b] > 0.0 ? signal[b] / (ssum[b] / wsum) : 0.0;
      }
      if (it < kPkIter) slopes(kmean, p, &neff);
    }
  }
  for (int b = 0; b < nb; ++b) {
    k_out[b] = kmean[b];
    p_out[b] = p[b];
    if (praw_out) praw_out[b] = praw[b];
  }
  return SDPM_OK;
}

}  // namespace sdpm
