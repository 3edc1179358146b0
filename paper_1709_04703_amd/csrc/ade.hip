// The paper's alternating-direction explicit (ADE) integrator of the gravity
// diffusion equation (Sec. 2.1 Eq. 4, Sec. 2.3).  One Saul'yev sweep of a
// half sub-step updates every cell of the active box in place,
//   (1 + 3 lam) phi_c' = (1 - 3 lam) phi_c + lam (S6 - f_c),
// lam = 1 / (kappa h^2), f = S h^2 delta, S6 the sum of the six neighbours'
// current values, visiting the cells in lexicographic order (forward: z, y,
// x increasing; backward: all decreasing), so that a neighbour visited
// earlier contributes its new value and one visited later its old value.
// The first half sub-step of a time step sweeps forward, the second
// backward (two consecutive steps in alternate directions).
//
// Parallel form.  Number the rows (j, k) of the box by their distance from
// the sweep's starting corner, jj + kk.  A row reads the rows (j -+ 1, k)
// and (j, k -+ 1): those visited before it lie on diagonal jj + kk - 1, those
// after it on jj + kk + 1, and so do the periodic wrap-around rows (a row at
// the far end of an axis is one diagonal step of n - 1 away, on the side of
// the visiting order).  So all rows of one diagonal can be updated in place
// by one launch, diagonals in order: every row then finds its earlier
// neighbours new and its later ones old, as in the sequential sweep.
// Within a row the cell t (counted along the sweep) obeys
//   u_t = c_t + a u_{t-1},   a = lam / (1 + 3 lam),
// with c_t holding the old centre, the later x neighbour, the four row
// neighbours and the source.  One wave owns a row: each lane computes the
// c_t of L consecutive cells, a scan of affine maps across the 64 lanes
// carries the recurrence, and each lane then writes its cells.  On the
// periodic mesh the later x neighbour of the row's last cell is its first
// cell, already new: its c_t is corrected with the first cell's new value
// before the scan.
#include <algorithm>

#include "internal.h"

namespace sdpm {
namespace {

constexpr int kAdeRowsPerBlock = 4;   // one row per wave, 4 waves per workgroup

template <int L, bool FWD>
__global__ void __launch_bounds__(256)
k_ade_diag(double* __restrict__ phi, const double* __restrict__ f, int n, Box b, int periodic,
           double lam, int d, int g0) {
  // workgroup g handles rows jj = 4 g .. 4 g + 3 of every diagonal, so a row
  // and its neighbour of the previous diagonal share a workgroup id and
  // therefore an XCD; groups below the diagonal's first row return at once
  if ((int)blockIdx.x < g0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = b.hi[0] - b.lo[0] + 1, ny = b.hi[1] - b.lo[1] + 1, nz = b.hi[2] - b.lo[2] + 1;
  const int jj = (int)blockIdx.x * kAdeRowsPerBlock + wave, kk = d - jj;
  if (jj >= ny || kk < 0 || kk >= nz) return;   // uniform over the wave
  const int m = n - 1;
  const int j = FWD ? b.lo[1] + jj : b.hi[1] - jj;
  const int k = FWD ? b.lo[2] + kk : b.hi[2] - kk;
  const int jm = periodic ? (j - 1) & m : j - 1, jp = periodic ? (j + 1) & m : j + 1;
  const int km = periodic ? (k - 1) & m : k - 1, kp = periodic ? (k + 1) & m : k + 1;
  const int64_t row = ((int64_t)k * n + j) * n;
  const int64_t rjm = ((int64_t)k * n + jm) * n, rjp = ((int64_t)k * n + jp) * n;
  const int64_t rkm = ((int64_t)km * n + j) * n, rkp = ((int64_t)kp * n + j) * n;
  constexpr int dir = FWD ? 1 : -1;
  const int i_first = FWD ? b.lo[0] : b.hi[0];
  const double inv = 1.0 / (1.0 + 3.0 * lam);
  const double co = 1.0 - 3.0 * lam;
  const double a = lam * inv;
  // the value before the first cell: the frozen exterior, or on the periodic
  // mesh the row's other end (not yet visited: old)
  const int i_before = periodic ? (i_first - dir) & m : i_first - dir;
  const double u_before = phi[row + i_before];
  const double first_old = phi[row + i_first];
  double c[L];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int t = lane * L + q;
    c[q] = 0.0;
    if (t < nx) {
      const int i = i_first + dir * t;
      const int in = periodic ? (i + dir) & m : i + dir;
      const double s = phi[row + in] + phi[rjm + i] + phi[rjp + i] + phi[rkm + i] + phi[rkp + i];
      c[q] = (co * phi[row + i] + lam * (s - f[row + i])) * inv;
    }
  }
  if (periodic) {
    // the last cell's later x neighbour is the first cell, new by now
    const double u_first = __shfl(c[0] + a * u_before, 0, 64);
#pragma unroll
    for (int q = 0; q < L; ++q)
      if (lane * L + q == nx - 1) c[q] += a * (u_first - first_old);
  }
  // this lane's cells as one affine map u_in -> A u_in + B
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int q = 0; q < L; ++q)
    if (lane * L + q < nx) {
      B = a * B + c[q];
      A *= a;
    }
  // inclusive scan over the lanes: (A, B) after (A', B') is (A A', A B' + B)
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double Ap = __shfl_up(A, off, 64), Bp = __shfl_up(B, off, 64);
    if (lane >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  double Ae = __shfl_up(A, 1, 64), Be = __shfl_up(B, 1, 64);
  if (lane == 0) Ae = 1.0, Be = 0.0;
  double u = Ae * u_before + Be;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int t = lane * L + q;
    if (t < nx) {
      u = a * u + c[q];
      phi[row + i_first + dir * t] = u;
    }
  }
}

template <int L>
void ade_diagonals(double* phi, const double* f, int n, const Box& b, int periodic, double lam,
                   bool forward, hipStream_t st) {
  const int ny = b.hi[1] - b.lo[1] + 1, nz = b.hi[2] - b.lo[2] + 1;
  for (int d = 0; d <= ny + nz - 2; ++d) {
    const int jlo = std::max(0, d - nz + 1), jhi = std::min(d, ny - 1);
    const unsigned grid = (unsigned)(jhi / kAdeRowsPerBlock + 1);
    const int g0 = jlo / kAdeRowsPerBlock;
    if (forward)
      hipLaunchKernelGGL((k_ade_diag<L, true>), dim3(grid), dim3(256), 0, st, phi, f, n, b,
                         periodic, lam, d, g0);
    else
      hipLaunchKernelGGL((k_ade_diag<L, false>), dim3(grid), dim3(256), 0, st, phi, f, n, b,
                         periodic, lam, d, g0);
  }
}

}  // namespace

void launch_ade_sweep(double* phi, const double* f, int n, const Box& b, bool periodic, double lam,
                      bool forward, hipStream_t st) {
  const int nx = b.hi[0] - b.lo[0] + 1;
  const int per = periodic ? 1 : 0;
  prof_begin(st, K_ADE);
  if (nx <= 64)
    ade_diagonals<1>(phi, f, n, b, per, lam, forward, st);
  else if (nx <= 128)
    ade_diagonals<2>(phi, f, n, b, per, lam, forward, st);
  else if (nx <= 256)
    ade_diagonals<4>(phi, f, n, b, per, lam, forward, st);
  else if (nx <= 512)
    ade_diagonals<8>(phi, f, n, b, per, lam, forward, st);
  else if (nx <= 1024)
    ade_diagonals<16>(phi, f, n, b, per, lam, forward, st);
  else
    ade_diagonals<32>(phi, f, n, b, per, lam, forward, st);
  // read phi and f, write phi once per cell
  prof_end(st, K_ADE, 24.0 * box_cells(b));
}

}  // namespace sdpm
