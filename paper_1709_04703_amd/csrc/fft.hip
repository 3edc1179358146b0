// Exact periodic solve of the mesh equation (Lap_h - kappa h^2) phi = rhs by
// FFT: the standard particle-mesh Poisson solver the paper compares against
// (Sec. 2.4), here also for kappa > 0 (the implicit half sub-step of
// Sec. 2.1 Eq. 4).  The 7-point operator is diagonal in Fourier space with
// symbol -(s(kx) + s(ky) + s(kz)) - kappa h^2, s(k) = 2 - 2 cos(2 pi k / n);
// the k = 0 mode of the singular periodic Poisson problem (kappa = 0) is set
// to zero (zero-mean potential).  Transforms are hipFFT FP64 real-to-complex
// and complex-to-real plans whose work area lives in the caller's workspace;
// the division by the symbol (and the 1 / n^3 of the inverse transform) is
// one pass over the half spectrum.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.h"

namespace sdpm {
namespace {

// C[k][j][i] for i <= n / 2 (hermitian half), divided by the symbol and n^3
__global__ void __launch_bounds__(256)
k_fft_divide(hipfftDoubleComplex* __restrict__ c, const double* __restrict__ s, int n,
             double kappa_h2, double inv_n3) {
  const int hx = n / 2 + 1;
  const int64_t total = (int64_t)n * n * hx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % hx);
    const int64_t r = q / hx;
    const int j = (int)(r % n), k = (int)(r / n);
    const double sym = -(s[i] + s[j] + s[k]) - kappa_h2;
    const double g = (sym != 0.0) ? inv_n3 / sym : 0.0;
    hipfftDoubleComplex v = c[q];
    v.x *= g;
    v.y *= g;
    c[q] = v;
  }
}

}  // namespace

size_t fft_complex_bytes(int n) { return (size_t)n * n * (n / 2 + 1) * sizeof(hipfftDoubleComplex); }

int fft_init(FftPlan* p, int n, void* complex_buf, void* work, size_t work_bytes, double* sym_dev,
             hipStream_t st, char* msg, size_t len) {
  p->n = n;
  p->c = complex_buf;
  p->sym = sym_dev;
  size_t ws_fwd = 0, ws_inv = 0;
  hipfftHandle fwd = 0, inv = 0;
  if (hipfftCreate(&fwd) != HIPFFT_SUCCESS) {
    snprintf(msg, len, "hipfftCreate failed");
    return SDPM_EHIP;
  }
  p->fwd = (void*)fwd;   // released by fft_destroy on every later failure
  if (hipfftCreate(&inv) != HIPFFT_SUCCESS) {
    snprintf(msg, len, "hipfftCreate failed");
    return SDPM_EHIP;
  }
  p->inv = (void*)inv;
  if (hipfftSetAutoAllocation(fwd, 0) != HIPFFT_SUCCESS ||
      hipfftSetAutoAllocation(inv, 0) != HIPFFT_SUCCESS ||
      hipfftMakePlan3d(fwd, n, n, n, HIPFFT_D2Z, &ws_fwd) != HIPFFT_SUCCESS ||
      hipfftMakePlan3d(inv, n, n, n, HIPFFT_Z2D, &ws_inv) != HIPFFT_SUCCESS) {
    snprintf(msg, len, "hipFFT plan creation failed for %d^3", n);
    return SDPM_EHIP;
  }
  if (ws_fwd > work_bytes || ws_inv > work_bytes) {
    snprintf(msg, len, "hipFFT needs a %zu-byte work area, the workspace holds %zu",
             std::max(ws_fwd, ws_inv), work_bytes);
    return SDPM_ENOMEM;
  }
  if (hipfftSetWorkArea(fwd, work) != HIPFFT_SUCCESS ||
      hipfftSetWorkArea(inv, work) != HIPFFT_SUCCESS ||
      hipfftSetStream(fwd, st) != HIPFFT_SUCCESS || hipfftSetStream(inv, st) != HIPFFT_SUCCESS) {
    snprintf(msg, len, "hipFFT work area / stream setup failed");
    return SDPM_EHIP;
  }
  std::vector<double> s(n);
  for (int k = 0; k < n; ++k) s[k] = 2.0 - 2.0 * std::cos(2.0 * M_PI * k / n);
  if (hipMemcpyAsync(sym_dev, s.data(), n * sizeof(double), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    snprintf(msg, len, "copy of the FFT symbol table failed");
    return SDPM_EHIP;
  }
  return SDPM_OK;
}

void fft_destroy(FftPlan* p) {
  if (p->fwd) hipfftDestroy((hipfftHandle)p->fwd);
  if (p->inv) hipfftDestroy((hipfftHandle)p->inv);
  p->fwd = p->inv = nullptr;
}

int fft_solve(const FftPlan& p, const double* rhs, double* phi, double kappa_h2, hipStream_t st) {
  const int n = p.n;
  const double cells = (double)n * n * n;
  auto* c = (hipfftDoubleComplex*)p.c;
  prof_begin(st, K_FFT);
  const hipfftResult r1 = hipfftExecD2Z((hipfftHandle)p.fwd, (hipfftDoubleReal*)rhs, c);
  prof_end(st, K_FFT, 16.0 * cells);   // read rhs, write the half spectrum
  if (r1 != HIPFFT_SUCCESS) return SDPM_EHIP;
  const int64_t half = (int64_t)n * n * (n / 2 + 1);
  prof_begin(st, K_FFT_DIVIDE);
  hipLaunchKernelGGL(k_fft_divide, dim3((unsigned)std::min<int64_t>((half + 255) / 256, 65536)),
                     dim3(256), 0, st, c, p.sym, n, kappa_h2, 1.0 / cells);
  prof_end(st, K_FFT_DIVIDE, 32.0 * (double)half);
  prof_begin(st, K_FFT);
  const hipfftResult r2 = hipfftExecZ2D((hipfftHandle)p.inv, c, (hipfftDoubleReal*)phi);
  prof_end(st, K_FFT, 16.0 * cells);
  return r2 == HIPFFT_SUCCESS ? SDPM_OK : SDPM_EHIP;
}

}  // namespace sdpm
