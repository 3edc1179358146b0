// Re-sort of the active particles: a 32-bit key per particle (the Morton
// code of its block of 2^shift cells per axis, then its cell row inside the
// block: z, then y), a stable LSD radix sort of (key, index) pairs with 8-bit
// digits, and a gather of the SoA particle arrays into sorted order.  Inside
// a row the particles keep their previous order.  The
// physics of a step does not depend on particle order (the deposit is exact
// integer arithmetic, every other pass is per particle, compaction is
// stable); the sort only makes neighbouring particles touch neighbouring
// cells, which the LDS-privatised deposit and the interpolation exploit.
//
// Radix pass: (1) each workgroup histograms the digit of its kChunk keys in
// LDS, (2) a device-wide exclusive scan over the digit-major table gives
// every (digit, workgroup) its output base, (3) each workgroup scatters its
// keys in order: the rank among equal digits inside a wavefront comes from
// 8 ballots (one per digit bit), wavefronts and rounds are chained through
// per-digit counters in LDS, so the pass is stable.
#include "internal.h"

namespace sdpm {
namespace {

constexpr int kDigits = 256;

__device__ inline uint32_t spread3(uint32_t v) {
  // insert two zero bits between the low 10-11 bits of v
  v &= 0x7ff;
  v = (v | (v << 16)) & 0x070000ff;
  v = (v | (v << 8)) & 0x0700f00f;
  v = (v | (v << 4)) & 0x430c30c3;
  v = (v | (v << 2)) & 0x49249249;
  return v;
}

__global__ void __launch_bounds__(256)
k_morton_keys(const double* __restrict__ x0, const double* __restrict__ x1,
              const double* __restrict__ x2, int64_t n, double inv_h, int ng, int shift,
              uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  int c[3];
  const double xs[3] = {x0[q], x1[q], x2[q]};
  for (int d = 0; d < 3; ++d) {
    double v = floor(xs[d] * inv_h);
    v = v < 0.0 ? 0.0 : (v > ng - 1 ? ng - 1 : v);   // NaN -> ng - 1: order only
    c[d] = (int)v;
  }
  const uint32_t in = (uint32_t)((1 << shift) - 1);
  const uint32_t block = spread3((uint32_t)(c[0] >> shift)) | (spread3((uint32_t)(c[1] >> shift)) << 1) |
                         (spread3((uint32_t)(c[2] >> shift)) << 2);
  key[q] = (block << (2 * shift)) | (((uint32_t)c[2] & in) << shift) | ((uint32_t)c[1] & in);
  val[q] = (uint32_t)q;
}

// First sorted index of each block (Morton index m): the lower bound of its
// first key m << 2 shift in the sorted keys; start[nblk] = n.
__global__ void __launch_bounds__(256)
k_block_starts(const uint32_t* __restrict__ key, int64_t n, int shift, int64_t nblk,
               int64_t* __restrict__ start) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m > nblk) return;
  if (m == nblk) {
    start[m] = n;
    return;
  }
  const uint32_t target = (uint32_t)m << (2 * shift);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  start[m] = lo;
}

__global__ void __launch_bounds__(256)
k_radix_hist(const uint32_t* __restrict__ key, int64_t n, int bit, int nblocks,
             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kDigits];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int u = 0; u < kChunk / 256; ++u) {
    const int64_t q = base + u * 256 + tid;
    if (q < n) atomicAdd(&h[(key[q] >> bit) & 0xff], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = h[tid];
}

template <bool HAS_VAL>
__global__ void __launch_bounds__(256)
k_radix_scatter(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val, int64_t n,
                int bit, int nblocks, const uint32_t* __restrict__ base_tab,
                uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
  __shared__ uint32_t whist[4][kDigits];
  __shared__ uint32_t run[kDigits];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  run[tid] = base_tab[(int64_t)tid * nblocks + blockIdx.x];
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  for (int u = 0; u < kChunk / 256; ++u) {
    const int64_t q = base + u * 256 + tid;
    const bool valid = q < n;
    const uint32_t k = valid ? key[q] : 0u;
    const uint32_t d = (k >> bit) & 0xff;
    for (int w = 0; w < 4; ++w) whist[w][tid] = 0;
    __syncthreads();
    // lanes of this wave holding the same digit
    unsigned long long same = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(same & lt);
    if (valid && rank == 0) whist[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t off = run[d];
      for (int w = 0; w < wave; ++w) off += whist[w][d];
      const uint32_t dst = off + rank;
      key_out[dst] = k;
      if (HAS_VAL) val_out[dst] = val[q];
    }
    __syncthreads();
    run[tid] += whist[0][tid] + whist[1][tid] + whist[2][tid] + whist[3][tid];
    __syncthreads();
  }
}

// device-wide exclusive scan of uint32 (three kernels)
constexpr int kScanSeg = 4096;

__global__ void __launch_bounds__(256)
k_scan_seg_sum(const uint32_t* __restrict__ a, int64_t n, uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[4];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanSeg;
  uint32_t s = 0;
  for (int u = 0; u < kScanSeg / 256; ++u) {
    const int64_t q = base + u * 256 + tid;
    if (q < n) s += a[q];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void __launch_bounds__(1024) k_scan_parts(uint32_t* __restrict__ part, int64_t np) {
  __shared__ uint32_t sh[1024];
  const int tid = threadIdx.x;
  const int64_t per = (np + 1023) / 1024;
  const int64_t b0 = tid * per, b1 = min(np, b0 + per);
  uint32_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += part[b];
  sh[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  uint32_t run = tid ? sh[tid - 1] : 0u;
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = part[b];
    part[b] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(256)
k_scan_apply(uint32_t* __restrict__ a, int64_t n, const uint32_t* __restrict__ part) {
  __shared__ uint32_t wtot[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanSeg;
  uint32_t run = part[blockIdx.x];
  for (int u = 0; u < kScanSeg / 256; ++u) {
    const int64_t q = base + u * 256 + tid;
    const uint32_t v = q < n ? a[q] : 0u;
    // inclusive wave scan
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    uint32_t woff = 0;
    for (int w = 0; w < wave; ++w) woff += wtot[w];
    if (q < n) a[q] = run + woff + x - v;
    run += wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
  }
}

template <typename PT>
__global__ void __launch_bounds__(256)
k_gather(ParticleArgs pa, const uint32_t* __restrict__ perm, double* __restrict__ sx0,
         double* __restrict__ sx1, double* __restrict__ sx2, PT* __restrict__ sp0,
         PT* __restrict__ sp1, PT* __restrict__ sp2, uint32_t* __restrict__ sid) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= pa.n) return;
  const uint32_t s = perm[q];
  sx0[q] = pa.x[0][s];
  sx1[q] = pa.x[1][s];
  sx2[q] = pa.x[2][s];
  sp0[q] = ((const PT*)pa.p[0])[s];
  sp1[q] = ((const PT*)pa.p[1])[s];
  sp2[q] = ((const PT*)pa.p[2])[s];
  sid[q] = pa.id[s];
}

void device_scan(uint32_t* a, int64_t n, uint32_t* part, hipStream_t st) {
  const int64_t np = (n + kScanSeg - 1) / kScanSeg;
  hipLaunchKernelGGL(k_scan_seg_sum, dim3((unsigned)np), dim3(256), 0, st, a, n, part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, st, part, np);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)np), dim3(256), 0, st, a, n, part);
}

}  // namespace

size_t sort_scratch_bytes(int64_t capacity) {
  const int64_t nb = (capacity + kChunk - 1) / kChunk + 1;
  const int64_t tab = nb * kDigits;
  const int64_t np = (tab + kScanSeg - 1) / kScanSeg + 1;
  return (size_t)(4 * capacity + tab + np) * sizeof(uint32_t) + 4 * 256;
}

template <typename PT>
void launch_morton_sort(const ParticleArgs& pa, int ng, double box, int shift, void* sort_scratch,
                        void* particle_scratch, int64_t* block_start, hipStream_t st) {
  const int64_t n = pa.n;
  if (n <= 1) return;
  const int64_t nb = (n + kChunk - 1) / kChunk;
  const int64_t tab = nb * kDigits;
  uint32_t* k0 = (uint32_t*)sort_scratch;
  uint32_t* v0 = k0 + n;
  uint32_t* k1 = v0 + n;
  uint32_t* v1 = k1 + n;
  uint32_t* hist = v1 + n;
  uint32_t* part = hist + tab;
  int lg = 0;
  while ((1 << lg) < ng) ++lg;
  const int bits = 3 * (lg - shift) + 2 * shift;
  const unsigned gp = (unsigned)((n + 255) / 256);
  prof_begin(st, K_SORT);
  hipLaunchKernelGGL(k_morton_keys, dim3(gp), dim3(256), 0, st, pa.x[0], pa.x[1], pa.x[2], n,
                     (double)ng / box, ng, shift, k0, v0);
  for (int bit = 0; bit < bits; bit += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(256), 0, st, k0, n, bit, (int)nb, hist);
    device_scan(hist, tab, part, st);
    hipLaunchKernelGGL((k_radix_scatter<true>), dim3((unsigned)nb), dim3(256), 0, st, k0, v0, n, bit,
                       (int)nb, hist, k1, v1);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  if (block_start) {
    const int64_t nb1 = ng >> shift, nblk = nb1 * nb1 * nb1;
    hipLaunchKernelGGL(k_block_starts, dim3((unsigned)((nblk + 256) / 256)), dim3(256), 0, st, k0, n,
                       shift, nblk, block_start);
  }
  const int passes = (bits + 7) / 8;
  prof_end(st, K_SORT, (double)n * (8.0 + passes * (4.0 + 16.0)));
  char* s = (char*)particle_scratch;
  double* sx0 = (double*)s;
  double* sx1 = sx0 + n;
  double* sx2 = sx1 + n;
  PT* sp0 = (PT*)(sx2 + n);
  PT* sp1 = sp0 + n;
  PT* sp2 = sp1 + n;
  uint32_t* sid = (uint32_t*)(sp2 + n);
  const double pbytes = (24.0 + 3.0 * sizeof(PT) + 4.0) * n;
  prof_begin(st, K_GATHER);
  hipLaunchKernelGGL(k_gather<PT>, dim3(gp), dim3(256), 0, st, pa, v0, sx0, sx1, sx2, sp0, sp1, sp2,
                     sid);
  prof_end(st, K_GATHER, 2.0 * pbytes + 4.0 * n);
  prof_begin(st, K_COPY);
  for (int d = 0; d < 3; ++d) {
    (void)hipMemcpyAsync(pa.x[d], sx0 + d * n, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(pa.p[d], sp0 + d * n, n * sizeof(PT), hipMemcpyDeviceToDevice, st);
  }
  (void)hipMemcpyAsync(pa.id, sid, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  prof_end(st, K_COPY, 2.0 * pbytes);
}
template void launch_morton_sort<float>(const ParticleArgs&, int, double, int, void*, void*,
                                        int64_t*, hipStream_t);
template void launch_morton_sort<double>(const ParticleArgs&, int, double, int, void*, void*,
                                         int64_t*, hipStream_t);

}  // namespace sdpm
