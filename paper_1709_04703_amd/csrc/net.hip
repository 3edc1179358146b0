// Learned warm start for the multigrid solve: a 5-layer 3x3x3 convolution
// net with 16 channels (ReLU between layers, periodic padding), BF16 weights
// and activations, FP32 accumulation on the matrix cores of gfx950.
//
// Each layer is an implicit GEMM over taps t:  Out^T (16 co x voxels) +=
// W_t^T (16 co x 16 ci) * In_t^T (16 ci x voxels).  Activations are stored
// channels-last (16 BF16 = 32 B per voxel), so a lane's B fragment (8 or 4
// channels of one voxel) is one 16- or 8-byte read and its D fragment (4
// channels of one voxel) one 8-byte write.  MFMA lane layouts (64 lanes,
// g = lane / 16, r = lane % 16): 16x16x16 A[r][4g..4g+3], B[4g..4g+3][r];
// 16x16x32 A[r][8g..8g+7], B[8g..8g+7][r]; both D[4g..4g+3][r].
//
// The data gradient of a layer is the same kernel with the taps mirrored and
// the channel roles swapped (BACKWARD flag); the weight gradient reduces
// In^T * G over voxels on the matrix cores, per workgroup, then in a fixed
// order over workgroups (deterministic).
#include <cmath>

#include "internal.h"

namespace sdpm {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNC = 16;                 // channels
constexpr int kCTY = 4, kCTZ = 8;             // weight-gradient tile: 4 rows, 8 planes

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;       // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                           // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline int64_t vox(int i, int j, int k, int n) { return ((int64_t)k * n + j) * n + i; }

// ---------------------------------------------------------------- forward
// flags: 1 ReLU, 2 FP32 output of channel 0 only, 4 backward-data (mirrored
// taps, swapped channels, no bias), 8 multiply by [mask > 0].
//
// v_mfma_f32_16x16x32_bf16 (K = 32: two taps of 16 input channels at once;
// gfx950 runs it at twice the rate of the K = 16 form).  Lane layout (g =
// lane / 16, r = lane % 16): A[r][8g .. 8g+7], B[8g .. 8g+7][r],
// D[4g .. 4g+3][r].  Taps are paired along x: one MFMA takes dx = -1 (k < 16)
// and dx = 0 (k >= 16) of an input row, a second dx = +1 (k < 16; the other
// half has zero weights).  A workgroup walks kZB blocks of kCZ planes; for
// each it holds the input voxels (64 + 2) x (kCY + 2) x (kCZ + 2) in an LDS
// ring of kBZ planes (consecutive blocks share two planes, so a block loads
// kCZ new ones); each of its 4 waves owns 16 output voxels in x for all
// kCY x kCZ output rows and reuses every input-row fragment it loads for the
// (up to 9) output rows that row feeds.  The weights stay in registers for
// all blocks.
typedef short bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kCY = 4, kCZ = 4;                  // output rows per block (y, z)
constexpr int kZB = 8;                           // z blocks per workgroup (weights loaded once)
constexpr int kBX = 64 + 2, kBY = kCY + 2, kBZ = kCZ + 2;

template <int FLAGS>
__global__ void __launch_bounds__(256)
k_conv(int n, const uint16_t* __restrict__ in, const float* __restrict__ w,
       const float* __restrict__ bias, const uint16_t* __restrict__ mask, void* __restrict__ out) {
  constexpr bool RELU = FLAGS & 1, OUT0 = FLAGS & 2, BWD = FLAGS & 4, MASK = FLAGS & 8;
  __shared__ __attribute__((aligned(16))) uint16_t blk[kBZ][kBY][kBX][kNC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15, hi = g >> 1, cg = g & 1;
  const int m = n - 1;
  const int gx = (n + 63) / 64, gy = n / kCY;
  const int bx = blockIdx.x % gx, by = (blockIdx.x / gx) % gy, bz = blockIdx.x / (gx * gy);
  const int x0 = bx * 64, y0 = by * kCY;
  // weight fragments per (dy, dz): a01 = taps dx = -1 (k < 16), dx = 0 (k >= 16);
  // a2 = tap dx = +1 (k < 16), zero for k >= 16.  Element j of lane (g, r):
  // input channel 8 cg + j, output channel r.
  bf16x8 a01[9], a2[9];
#pragma unroll
  for (int yz = 0; yz < 9; ++yz) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ci = 8 * cg + j;
      const int t01 = yz * 3 + (hi ? 1 : 0), t2 = yz * 3 + 2;
      const float v01 = BWD ? w[((26 - t01) * kNC + r) * kNC + ci] : w[(t01 * kNC + ci) * kNC + r];
      const float v2 = BWD ? w[((26 - t2) * kNC + r) * kNC + ci] : w[(t2 * kNC + ci) * kNC + r];
      a01[yz][j] = (short)f2bf(v01);
      a2[yz][j] = hi ? (short)0 : (short)f2bf(v2);
    }
  }
  float bq[4] = {0.f, 0.f, 0.f, 0.f};
  if (!BWD && bias) {
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[q] = bias[4 * g + q];
  }
  for (int zb = 0; zb < kZB; ++zb) {
  const int z0 = (bz * kZB + zb) * kCZ;
  if (z0 >= n) break;
  __syncthreads();                               // the planes to overwrite are consumed
  // input plane z0 - 1 + pz sits in ring slot (kCZ zb + pz) % kBZ; planes
  // pz < 2 were loaded with the previous block.  16 bytes per load.
  const int pz0 = zb == 0 ? 0 : 2;
  for (int c = tid; c < (kBZ - pz0) * kBY * kBX * 2; c += 256) {
    const int half = c & 1, v = c >> 1;
    const int px = v % kBX, py = (v / kBX) % kBY, pz = pz0 + v / (kBX * kBY);
    const int xx = (x0 - 1 + px) & m, yy = (y0 - 1 + py) & m, zz = (z0 - 1 + pz) & m;
    ((uint4*)&blk[(kCZ * zb + pz) % kBZ][py][px][0])[half] =
        ((const uint4*)(in + vox(xx, yy, zz, n) * kNC))[half];
  }
  f32x4 acc[kCZ][kCY];
#pragma unroll
  for (int a = 0; a < kCZ; ++a)
#pragma unroll
    for (int b = 0; b < kCY; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();
  // output voxel x0 + 16 wave + r reads block column 16 wave + r + 1 + dx
  const int col = 16 * wave + r + 1;
#pragma unroll
  for (int pz = 0; pz < kBZ; ++pz) {
#pragma unroll
    for (int py = 0; py < kBY; ++py) {
      // F01: k < 16 from x - 1, k >= 16 from x; F2: x + 1 (both halves)
      const int sl = (kCZ * zb + pz) % kBZ;
      const bf16x8 f01 = *(const bf16x8*)&blk[sl][py][col - 1 + hi][8 * cg];
      const bf16x8 f2 = *(const bf16x8*)&blk[sl][py][col + 1][8 * cg];
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
        const int oz = pz - 1 - dz;            // output row fed with this tap
        if (oz < 0 || oz >= kCZ) continue;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          const int oy = py - 1 - dy;
          if (oy < 0 || oy >= kCY) continue;
          const int yz = (dz + 1) * 3 + (dy + 1);
          acc[oz][oy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a01[yz], f01, acc[oz][oy], 0, 0, 0);
          acc[oz][oy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[yz], f2, acc[oz][oy], 0, 0, 0);
        }
      }
    }
  }
  // D[co = 4g + q][voxel = r] of each output row
  const int x = (x0 + 16 * wave + r) & m;
#pragma unroll
  for (int oz = 0; oz < kCZ; ++oz) {
#pragma unroll
    for (int oy = 0; oy < kCY; ++oy) {
      const int64_t v = vox(x, (y0 + oy) & m, (z0 + oz) & m, n);
      float val[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float a = acc[oz][oy][q] + bq[q];
        if (RELU) a = a > 0.f ? a : 0.f;
        val[q] = a;
      }
      if (MASK) {
        const bf16x4 mk = *(const bf16x4*)(mask + v * kNC + 4 * g);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (!(bf2f((uint16_t)mk[q]) > 0.f)) val[q] = 0.f;
      }
      if (OUT0) {
        if (g == 0) ((float*)out)[v] = val[0];
      } else {
        bf16x4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (short)f2bf(val[q]);
        *(bf16x4*)((uint16_t*)out + v * kNC + 4 * g) = o;
      }
    }
  }
  }
}

// ---------------------------------------------------------- weight gradient
// dW[t][ci][co] = sum_v in[v + off_t][ci] g[v][co]; db[co] = sum_v g[v][co].
// MFMA: D (ci x co) += A (ci x 16 voxels) * B (16 voxels x co) with
// A[ci = r][k = 4g + q] = in[v_k + off_t][ci], B[k][co = r] = g[v_k][co].
// A workgroup covers gxw groups of 16 voxels in x, 4 rows, kCTZ planes; the
// 4 waves' partials are summed in LDS and written per workgroup.
constexpr int kWG = 27 * kNC * kNC + kNC;   // partial size per workgroup

__global__ void __launch_bounds__(256)
k_conv_wgrad(int n, const uint16_t* __restrict__ in, const uint16_t* __restrict__ gr,
             float* __restrict__ partial) {
  __shared__ float red[kWG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int m = n - 1;
  const int groups = n >= 64 ? 4 : n / 16;        // 16-voxel groups per row in a workgroup
  const int gx = n / (16 * groups), gy = n / kCTY;
  const int bx = blockIdx.x % gx, by = (blockIdx.x / gx) % gy, bz = blockIdx.x / (gx * gy);
  const int x0 = bx * 16 * groups, y = by * kCTY + wave, z0 = bz * kCTZ;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int z = z0; z < z0 + kCTZ && z < n; ++z) {
    for (int s = 0; s < groups; ++s) {
      const int xb = x0 + 16 * s + 4 * g;
      bf16x4 b;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint16_t gv = gr[vox(xb + q, y, z, n) * kNC + r];
        b[q] = (short)gv;
        bsum += bf2f(gv);
      }
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          a[q] = (short)in[vox((xb + q + dx) & m, (y + dy) & m, (z + dz) & m, n) * kNC + r];
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // sum the 4 waves: D[ci = 4g + q][co = r]
  for (int c = tid; c < kWG; c += 256) red[c] = 0.f;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(t * kNC + 4 * g + q) * kNC + r] += acc[t][q];
      // bias: the 4 lanes of equal r hold disjoint voxels; add them with
      // cross-lane shuffles, then one lane per channel updates LDS
      float bs = bsum;
      bs += __shfl_xor(bs, 16, 64);
      bs += __shfl_xor(bs, 32, 64);
      if (g == 0) red[27 * kNC * kNC + r] += bs;
    }
    __syncthreads();
  }
  float* dst = partial + (int64_t)blockIdx.x * kWG;
  for (int c = tid; c < kWG; c += 256) dst[c] = red[c];
}

__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float* __restrict__ partial, int nblocks, float* __restrict__ dw,
               float* __restrict__ db) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= kWG) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * kWG + c];
  if (c < 27 * kNC * kNC)
    dw[c] = s;
  else
    db[c - 27 * kNC * kNC] = s;
}

// ------------------------------------------------------------- inputs, loss
// act0[v] = (r[v] s_r, phi[v] s_phi, kap, 0, ...) in BF16.  RT / PT: input types;
// SPLIT: r stored colour-split; with a box, r outside it counts as zero.
template <typename RT, typename PT, bool SPLIT>
__global__ void __launch_bounds__(256)
k_net_prep(int n, const RT* __restrict__ r, const PT* __restrict__ phi, float s_r, float s_phi,
           float kap, Box b, int use_box, uint16_t* __restrict__ act0) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t V = (int64_t)n * n * n;
  if (v >= V) return;
  const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
  float rv = 0.f;
  const bool in_box = !use_box || (i >= b.lo[0] && i <= b.hi[0] && j >= b.lo[1] && j <= b.hi[1] &&
                                   k >= b.lo[2] && k <= b.hi[2]);
  if (in_box) {
    const int64_t hc = (int64_t)n * n * (n >> 1);
    const int64_t ri = SPLIT ? ((int64_t)((i + j + k) & 1) * hc + ((int64_t)k * n + j) * (n >> 1) + (i >> 1)) : v;
    rv = (float)r[ri] * s_r;
  }
  const float pv = (float)phi[v] * s_phi;
  uint4 o0, o1;
  o0.x = (uint32_t)f2bf(rv) | ((uint32_t)f2bf(pv) << 16);
  o0.y = (uint32_t)f2bf(kap);
  o0.z = o0.w = 0u;
  o1.x = o1.y = o1.z = o1.w = 0u;
  ((uint4*)(act0 + v * kNC))[0] = o0;
  ((uint4*)(act0 + v * kNC))[1] = o1;
}

// g[v] = (2 (out - tscale target) gscale, 0, ...) in BF16; partial sum of
// (out - tscale target)^2.
__global__ void __launch_bounds__(256)
k_net_loss(int64_t V, const float* __restrict__ out, const float* __restrict__ target, float tscale,
           float gscale, uint16_t* __restrict__ g, float* __restrict__ partial) {
  __shared__ float sh[4];
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float d = 0.f;
  if (v < V) {
    d = out[v] - target[v] * tscale;
    uint4 o0, o1;
    o0.x = (uint32_t)f2bf(2.f * d * gscale);
    o0.y = o0.z = o0.w = 0u;
    o1.x = o1.y = o1.z = o1.w = 0u;
    ((uint4*)(g + v * kNC))[0] = o0;
    ((uint4*)(g + v * kNC))[1] = o1;
  }
  float s = d * d;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void __launch_bounds__(256)
k_sum_partials(const float* __restrict__ partial, int np, float scale, float* __restrict__ out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int q = threadIdx.x; q < np; q += 256) s += partial[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// Adam on the FP32 master parameters; the input channels >= 2 of layer 0 and
// the output channels >= 1 of layer 4 stay zero.
__global__ void __launch_bounds__(256)
k_adam(int np, float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m1,
       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= np) return;
  const int per = 27 * kNC * kNC + kNC;
  const int l = q / per, o = q % per;
  bool frozen = false;
  if (o < 27 * kNC * kNC) {
    const int ci = (o / kNC) % kNC, co = o % kNC;
    frozen = (l == 0 && ci >= kNetInputs) || (l == 4 && co >= 1);
  } else {
    frozen = (l == 4 && o - 27 * kNC * kNC >= 1);
  }
  if (frozen) {
    p[q] = 0.f;
    return;
  }
  const float gq = grad[q];
  const float a = b1 * m1[q] + (1.f - b1) * gq;
  const float b = b2 * m2[q] + (1.f - b2) * gq * gq;
  m1[q] = a;
  m2[q] = b;
  p[q] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

int conv_blocks(int n) { return ((n + 63) / 64) * (n / kCY) * ((n / kCZ + kZB - 1) / kZB); }
int wgrad_blocks(int n) {
  const int groups = n >= 64 ? 4 : n / 16;
  return (n / (16 * groups)) * (n / kCTY) * ((n + kCTZ - 1) / kCTZ);
}

}  // namespace

bool net_size_ok(int n) { return n >= 16 && (n & (n - 1)) == 0; }

void launch_conv(int n, const uint16_t* in, const float* w, const float* bias, int flags,
                 const uint16_t* mask, void* out, hipStream_t st) {
  const dim3 g(conv_blocks(n));
  const double V = (double)n * n * n;
  prof_begin(st, K_CONV);
  switch (flags) {
    case 1: hipLaunchKernelGGL(k_conv<1>, g, dim3(256), 0, st, n, in, w, bias, mask, out); break;
    case 2: hipLaunchKernelGGL(k_conv<2>, g, dim3(256), 0, st, n, in, w, bias, mask, out); break;
    case 4: hipLaunchKernelGGL(k_conv<4>, g, dim3(256), 0, st, n, in, w, bias, mask, out); break;
    case 12: hipLaunchKernelGGL(k_conv<12>, g, dim3(256), 0, st, n, in, w, bias, mask, out); break;
    default: hipLaunchKernelGGL(k_conv<0>, g, dim3(256), 0, st, n, in, w, bias, mask, out); break;
  }
  // matrix-core work: 27 taps x 16 x 16 MACs per voxel
  prof_end(st, K_CONV, 2.0 * 27 * kNC * kNC * V);
}

size_t wgrad_scratch_bytes(int n) { return (size_t)wgrad_blocks(n) * kWG * sizeof(float); }

void launch_conv_wgrad(int n, const uint16_t* in, const uint16_t* g, float* dw, float* db,
                       float* scratch, hipStream_t st) {
  const int nb = wgrad_blocks(n);
  prof_begin(st, K_CONV_WGRAD);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(nb), dim3(256), 0, st, n, in, g, scratch);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((kWG + 255) / 256), dim3(256), 0, st, scratch, nb, dw, db);
  prof_end(st, K_CONV_WGRAD, 2.0 * 27 * kNC * kNC * (double)n * n * n);
}

template <typename RT, typename PT, bool SPLIT>
void launch_net_prep(int n, const RT* r, const PT* phi, float s_r, float s_phi, float kap,
                     const Box* box, uint16_t* act0, hipStream_t st) {
  const int64_t V = (int64_t)n * n * n;
  Box b{};
  if (box) b = *box;
  hipLaunchKernelGGL((k_net_prep<RT, PT, SPLIT>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0,
                     st, n, r, phi, s_r, s_phi, kap, b, box ? 1 : 0, act0);
}
template void launch_net_prep<float, float, false>(int, const float*, const float*, float, float,
                                                   float, const Box*, uint16_t*, hipStream_t);
template void launch_net_prep<float, double, true>(int, const float*, const double*, float, float,
                                                   float, const Box*, uint16_t*, hipStream_t);
template void launch_net_prep<double, double, true>(int, const double*, const double*, float, float,
                                                    float, const Box*, uint16_t*, hipStream_t);

// Net forward: act0 -> 4 hidden layers (ReLU, BF16) -> FP32 channel 0 in out.
void net_forward(int n, const float* params, const uint16_t* act0, uint16_t* a, uint16_t* b,
                 float* out, hipStream_t st) {
  const int per = 27 * kNC * kNC + kNC;
  const uint16_t* src = act0;
  uint16_t* bufs[2] = {a, b};
  for (int l = 0; l < 4; ++l) {
    const float* w = params + l * per;
    launch_conv(n, src, w, w + 27 * kNC * kNC, 1, nullptr, bufs[l & 1], st);
    src = bufs[l & 1];
  }
  const float* w = params + 4 * per;
  launch_conv(n, src, w, w + 27 * kNC * kNC, 2, nullptr, out, st);
}

size_t net_train_scratch_bytes(int n) {
  const size_t V = (size_t)n * n * n;
  const size_t act = V * kNC * sizeof(uint16_t);
  const size_t np = 5 * (27 * kNC * kNC + kNC);
  return 6 * act + V * sizeof(float) + wgrad_scratch_bytes(n) + np * sizeof(float) +
         ((V + 255) / 256) * sizeof(float) + 4096;
}

// One training step on one sample: forward with stored activations, MSE loss
// against target, backward through every layer, Adam.  loss_out (device):
// mean squared error of this sample.
void net_train_step(int n, float* params, float* m1, float* m2, int step, float lr,
                    const uint16_t* act0, const float* target, float target_scale, void* scratch,
                    float* loss_out, hipStream_t st) {
  const size_t V = (size_t)n * n * n;
  const int per = 27 * kNC * kNC + kNC;
  const int np = 5 * per;
  char* s = (char*)scratch;
  uint16_t* acts[5];
  acts[0] = (uint16_t*)act0;
  for (int l = 1; l < 5; ++l) {
    acts[l] = (uint16_t*)s;
    s += V * kNC * sizeof(uint16_t);
  }
  uint16_t* ga = (uint16_t*)s;
  s += V * kNC * sizeof(uint16_t);
  uint16_t* gb = (uint16_t*)s;
  s += V * kNC * sizeof(uint16_t);
  float* out = (float*)s;
  s += V * sizeof(float);
  float* wpart = (float*)s;
  s += wgrad_scratch_bytes(n);
  float* grad = (float*)s;
  s += (size_t)np * sizeof(float);
  float* lpart = (float*)s;
  for (int l = 0; l < 4; ++l) {
    const float* w = params + l * per;
    launch_conv(n, acts[l], w, w + 27 * kNC * kNC, 1, nullptr, acts[l + 1], st);
  }
  launch_conv(n, acts[4], params + 4 * per, params + 4 * per + 27 * kNC * kNC, 2, nullptr, out, st);
  const unsigned nbl = (unsigned)((V + 255) / 256);
  hipLaunchKernelGGL(k_net_loss, dim3(nbl), dim3(256), 0, st, (int64_t)V, out, target,
                     target_scale, 1.0f / (float)V, ga, lpart);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, lpart, (int)nbl, 1.0f / (float)V,
                     loss_out);
  uint16_t* gcur = ga;
  uint16_t* gnext = gb;
  for (int l = 4; l >= 0; --l) {
    float* dw = grad + l * per;
    launch_conv_wgrad(n, acts[l], gcur, dw, dw + 27 * kNC * kNC, wpart, st);
    if (l > 0) {
      // gradient into layer l's input, through the ReLU of layer l-1's output
      launch_conv(n, gcur, params + l * per, nullptr, 12, acts[l], gnext, st);
      uint16_t* tmp = gcur;
      gcur = gnext;
      gnext = tmp;
    }
  }
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, st, np, params, grad, m1, m2, lr,
                     b1, b2, 1e-8f, c1, c2);
}

}  // namespace sdpm
