// Internal declarations shared by the libsdpm translation units (not part of
// the C ABI).  Every kernel is written for gfx950: 64-lane wavefronts,
// 256-thread workgroups for the streaming kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/sdpm.h"

namespace sdpm {

constexpr int kMaxLevels = 12;
constexpr int kGateProbe = 8, kGateProbeMax = 256;   // solves skipped by the net gate
// host scalars: hpin[0..15] reduction results, [16..19] flags, [20] kept
// count, [kHostNorm ..] the ring of per-iteration residual norms
constexpr int kNormSlot = 16, kNormRing = 32, kHostNorm = 64, kHostScalars = 128;
// the four sums of a residual estimate (launch_correct_est), in dscal and hpin
constexpr int kEstSlot = 4;
// run-ahead of the outer iterations: at most kMaxAhead without a host wait,
// and only while the predicted norm exceeds kAheadMargin * threshold
constexpr int kMaxAhead = 16;
constexpr double kAheadMargin = 10.0;
// a further V-cycle in an outer iteration only while the cycles so far are
// predicted, with the factor per cycle measured in the last solve of the
// same kind, to leave the norm above kCycleMargin * threshold (a cycle too
// few costs a further outer iteration: its FP64 residual pass, a second
// estimating correction pass and a host wait, about 1.5 times a 512^3
// V-cycle, so the cycle is added once failing is about as likely as not)
// and their combined factor stays above kFloorMargin times the bound on the
// rounding floor of the correction; at most kMaxCyclesPerOuter cycles.
// Before any solve of that kind has measured the factor, its guess (0.1)
// only adds cycles while the prediction stays above kCycleMarginGuess times
// the threshold.
constexpr double kCycleMargin = 0.9;
constexpr double kCycleMarginGuess = 2.0;
constexpr int kMaxCyclesPerOuter = 4;
constexpr double kFloorMargin = 1.0;
constexpr int kHostLcCount = 120;      // host slot of the fixed-domain lightcone counter
constexpr int kCoarseMax = 16;        // coarsest multigrid level: at most 16^3 cells
constexpr int kBoxTx = 64;            // box kernels: 64 x 4 threads, KZ cells in z
constexpr int kBoxTy = 4;
constexpr int kBoxKz = 8;
constexpr int kChunk = 1024;          // particles per workgroup in the compaction passes
constexpr int kReduceSlots = 4;       // independent sums carried by one reduction

// Inclusive index box of one mesh level (axis order x, y, z).
struct Box {
  int lo[3];
  int hi[3];
};

// Logical workgroup of a 1-D launch: the hardware deals consecutive
// workgroup ids to the 8 XCDs in turn; this gives each XCD one contiguous run
// of logical ids, so work items that are neighbours in memory (Morton-ordered
// particles, neighbouring mesh tiles) share that XCD's L2.
__device__ inline int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t xcd = b & 7, slot = b >> 3;
  const int64_t per = nb >> 3, rem = nb & 7;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

__host__ __device__ inline int64_t lin(int i, int j, int k, int n) {
  return ((int64_t)k * n + j) * n + i;
}

inline int64_t box_cells(const Box& b) {
  return (int64_t)(b.hi[0] - b.lo[0] + 1) * (b.hi[1] - b.lo[1] + 1) * (b.hi[2] - b.lo[2] + 1);
}

// 1-D grid of box tiles (kBoxTx cells in x, kBoxTy rows, kBoxKz planes);
// kernels recover the tile with an XCD-aware remap of blockIdx.x.
inline dim3 box_grid(const Box& b) {
  const int nx = b.hi[0] - b.lo[0] + 1, ny = b.hi[1] - b.lo[1] + 1, nz = b.hi[2] - b.lo[2] + 1;
  return dim3((unsigned)(((nx + kBoxTx - 1) / kBoxTx) * ((ny + kBoxTy - 1) / kBoxTy) *
                         ((nz + kBoxKz - 1) / kBoxKz)));
}
// Same for kernels whose threads map to half-row (colour-split) indices.
inline dim3 half_grid(const Box& b) {
  const int hx = (b.hi[0] >> 1) - (b.lo[0] >> 1) + 1, ny = b.hi[1] - b.lo[1] + 1,
            nz = b.hi[2] - b.lo[2] + 1;
  return dim3((unsigned)(((hx + kBoxTx - 1) / kBoxTx) * ((ny + kBoxTy - 1) / kBoxTy) *
                         ((nz + kBoxKz - 1) / kBoxKz)));
}

// One multigrid level: `n` cells per axis (power of two), active box, and
// arrays of the correction e, the right-hand side r and a residual scratch t.
struct Level {
  int n;
  Box box;
  void* e;    // correction     } all three stored split by colour:
  void* r;    // right-hand side } red cells ((i+j+k) even) first, then black,
  void* t;    // residual        } each in row order with x index i >> 1
  void* e_alt;  // second correction array of the fused sweeps (FP32 levels of
                // at least kSweep4Min cells a side; else null): they read one
                // and write the other, and the two swap
};

// ---------------------------------------------------------------------------
// Host-side background cosmology (cosmology.cpp)
// ---------------------------------------------------------------------------
struct StepScalars {
  double dtau, a_half, s_half, kappa1_h2, kappa2_h2, r_lc_end, c_g;
};
double hubble_e(double a, double om, double ol);
double conformal_dtau(double a0, double a1, double om, double ol);
double conformal_midpoint(double a0, double a1, double om, double ol);
double lightcone_radius(double a, double om, double ol, double c_light);
StepScalars step_scalars(const sdpm_config& cfg, double a, double da);

// ---------------------------------------------------------------------------
// Launchers, mesh kernels (mesh.hip).  All enqueue on `st`.
// ---------------------------------------------------------------------------
template <typename T> void launch_fill(T* a, int n, const Box& b, T v, hipStream_t st);
// rhs = c_scale counts - c_off - kappa phi, ||rhs||^2 partials.  With chg
// (the extrapolated start): chg = apply ? (float)(chg_scale chg) : 0 and
// phi += chg, so chg then holds the change of phi since the rhs was formed.
void launch_rhs(const uint64_t* counts, double* phi, double* rhs, int n, const Box& b,
                double c_scale, double c_off, double kappa, float* chg, double chg_scale,
                bool apply, double* partial, int* nblocks, hipStream_t st);
template <typename T>
void launch_residual(const double* phi, const double* rhs, T* r_out, int n, const Box& b,
                     double kappa, double* partial, int* nblocks, hipStream_t st);
// phi += e (colour-split e); chg += e as well when chg is given.
// pending_scale != 0: a pending start d = (float)(pending_scale chg) is
// added first, phi = (phi + d) + e, chg = d + e.
template <typename T>
void launch_correct(double* phi, const T* e, float* chg, double pending_scale, int n,
                    const Box& b, hipStream_t st);
// launch_correct fused with an estimate of the next residual, r_old - A e
// (r_old: the residual the correction e solved for, colour-split T), in
// place of the FP64 residual pass; partial sums over *nblocks workgroups of
// the squares of the estimate, r_old, the new phi and e in slots 0..3.
template <typename T>
void launch_correct_est(double* phi, const T* e, const T* r_old, float* chg, double pending_scale,
                        double kappa, int n, const Box& b, double* partial, int* nblocks,
                        hipStream_t st);
// A pending start over the box: d = (float)(chg_scale chg), phi += d, chg = d.
void launch_apply_start(double* phi, float* chg, double chg_scale, int n, const Box& b,
                        hipStream_t st);
// The rhs pass fused with the first FP64 residual of a multigrid solve:
// rhs and r (colour-split T) with phi0 = phi + (float)(chg_scale chg) when
// apply (the start is then pending: phi and chg unchanged), else phi0 = phi
// and chg (when given) cleared; partial[0 .. nb) = rhs^2, partial[nb ..
// 2 nb) = r^2 sums.  With g3 the pass also writes the FP32 force mesh of
// phi (as launch_force_mesh with inv2h = 1 / 2h) over the same box.
// Returns false without launching when the box is narrower than the vector
// tiles.
template <typename T>
bool launch_rhs_residual(const uint64_t* counts, const double* phi, double* rhs, T* r_out,
                         float* chg, bool apply, double chg_scale, int n, const Box& b,
                         double c_scale, double c_off, double kappa, double* partial,
                         int* nblocks, hipStream_t st, float* g3 = nullptr, double inv2h = 0.0);

void launch_sum_phi(const double* phi, int n, const Box& b, double* partial, int* nblocks,
                    hipStream_t st);
void launch_add_const(double* phi, float* chg, int n, const Box& b, double v, hipStream_t st);
void launch_reduce_final(const double* partial, int nblocks, int nslots, double* out,
                         hipStream_t st);
// Exact periodic FFT solve of (Lap_h - kappa h^2) phi = rhs (fft.hip): FP64
// real-to-complex / complex-to-real plans on an n^3 mesh, half-spectrum
// buffer c, the 1-D symbol table sym (n values) on the device.
struct FftPlan {
  int n = 0;
  void* fwd = nullptr;
  void* inv = nullptr;
  void* c = nullptr;
  double* sym = nullptr;
};
size_t fft_complex_bytes(int n);
int fft_init(FftPlan* p, int n, void* complex_buf, void* work, size_t work_bytes, double* sym_dev,
             hipStream_t st, char* msg, size_t len);
void fft_destroy(FftPlan* p);
int fft_solve(const FftPlan& p, const double* rhs, double* phi, double kappa_h2, hipStream_t st);
// Power spectrum of particle positions (pk.hip; see sdpm_power_spectrum).
size_t pk_workspace_bytes(int n);
int power_spectrum(const double* const x[3], int64_t npart, double box, int n, int flags,
                   void* ws, hipStream_t st, double* k_out, double* p_out, double* praw_out,
                   int64_t* modes_out, char* msg, size_t len);
// One ADE sweep of phi over box b with source f (ade.hip).
void launch_ade_sweep(double* phi, const double* f, int n, const Box& b, bool periodic, double lam,
                      bool forward, hipStream_t st);
// One V-cycle for A_0 e = r_0; returns the level-0 buffer holding e.  With
// fine_start the cycle improves the e already on level 0 (a further cycle on
// the same r_0), else it starts from e = 0.  Levels with the fused sweeps
// swap e and e_alt.
template <typename T>
const T* vcycle(Level* lv, int nlev, double kappa, int pre, int post, int coarse_sweeps,
                bool periodic, bool fine_start, hipStream_t st);
// Whether a level of n cells a side takes the fused four-sweep kernel (FP32
// only; smaller levels run too few workgroups for it).
constexpr int kSweep4Min = 256;
// Four colour sweeps (red, black, red, black) of a periodic FP32 level of
// n^3 cells, n a power of two >= 64: with fused, one k_sweep4 pass from e
// (black colour; not read when first) into e_out (e_out == e allowed only
// when first); otherwise e copied to e_out (not when first) and four
// k_smooth_color_v4 launches in place on e_out.  With t (may be null) the
// red residual of the result goes to t's red half (inv_scale = 1 / scale,
// kappa = kappa h^2): in the fused pass instead of the red half of e_out,
// which it then leaves unwritten; otherwise by k_resid_red_v4.
// With box (may be null: the periodic whole mesh) the sweeps cover a
// frozen-exterior box that keeps at least one plane from every face of the
// mesh, e being zero outside it.
void launch_sweeps4(const float* e, float* e_out, const float* r, int n, float scale, float inv_diag,
                    bool first, bool fused, float* t, float inv_scale, float kappa, const Box* box,
                    hipStream_t st);

// ---------------------------------------------------------------------------
// Launchers, particle kernels (particles.hip).
// ---------------------------------------------------------------------------
struct ParticleArgs {
  double* x[3];
  void* p[3];
  uint32_t* id;
  int64_t n;
};
struct MeshMap {
  int ng;
  int frac_bits;
  int periodic;
  double box;         // L
  double scale;       // s = ng 2^B / L
  Box active;         // deposit / interpolation cells must lie inside
  int tsc;            // 0: CIC, 1: TSC assignment
  int block_shift;    // the re-sort's blocks: 2^block_shift cells per axis
};
// Fixed-point CIC / TSC deposit into counts, at the positions drifted by
// drift_coef p when drift != 0 (the drifted positions are not stored: the
// step's interpolation pass recomputes them).  flags[0] collects error bits.
template <typename PT>
void launch_drift_deposit(const ParticleArgs& pa, double drift_coef, int drift,
                          const MeshMap& mm, uint64_t* counts, uint32_t* flags, hipStream_t st);
// g3 (FP32, 3 per cell in natural order) = -grad Phi by central differences
// on the cells of box b (mesh.hip).
void launch_force_mesh(const double* phi, float* g3, int n, const Box& b, double inv2h,
                       hipStream_t st);
// Lightcone records of particles [first, first + count) (see sdpm.h): light
// = c dtau, disp = dtau / a1; written at out index out_first + q.
struct LcArgs {
  uint32_t* id;
  double* a;
  double* x[3];
  double* p[3];
};
template <typename PT>
void launch_lightcone(const ParticleArgs& pa, int64_t first, int64_t count, const double* x_obs,
                      double r1, double light, double disp, double a1, double da, const LcArgs& out,
                      int64_t out_first, hipStream_t st);
// Lightcone output on a fixed domain: marks of the particles outside radius
// sqrt(r2) at a step's start, then records of those outside at its end and
// not marked, in slots base + atomic counter (below capacity).
void launch_lc_mark(const ParticleArgs& pa, const double* x_obs, double r2, uint8_t* mark,
                    hipStream_t st);
template <typename PT>
void launch_lc_cross(const ParticleArgs& pa, const double* x_obs, double r2, double r,
                     double light, double disp, double a1, double da, const uint8_t* mark,
                     const LcArgs& out, int64_t base, int64_t capacity,
                     unsigned long long* counter, hipStream_t st);
// First drift (drift0_coef p, the positions the deposit used), force
// interpolation, kick and second drift of the active particles.  With g3 !=
// nullptr the force is interpolated from that mesh (made by
// launch_force_mesh), else from phi directly (FP64 differences).
template <typename PT>
void launch_interp_kick_drift(const ParticleArgs& pa, const double* phi, const float* g3,
                              const MeshMap& mm, double inv2h, double drift0_coef,
                              double kick_coef, double drift_coef, const double* x_obs, double r2,
                              int count_removed, uint32_t* removed_count, uint32_t* flags,
                              hipStream_t st);
void launch_interp_force(const ParticleArgs& pa, const double* phi, const MeshMap& mm,
                         double inv2h, double* g0, double* g1, double* g2, uint32_t* flags,
                         hipStream_t st);
// Stable partition of the first n particles: kept (d^2 <= r2) first.
// scratch must hold n particles; counts/offsets hold ceil(n / kChunk) entries.
// block_start (optional): the block deposit's table of nblk + 1 first
// indices, carried over to the compacted order.
template <typename PT>
void launch_compact(const ParticleArgs& pa, const double* x_obs, double r2, void* scratch,
                    uint32_t* block_counts, uint32_t* block_offsets, uint64_t* kept_total,
                    int64_t* block_start, int64_t nblk, hipStream_t st);

// Morton re-sort (sort.hip): sort_scratch holds sort_scratch_bytes(capacity),
// particle_scratch one particle set.  block_start (optional, (ng >> shift)^3
// + 1 entries): the first sorted index of each block in Morton order, the
// last entry n.
size_t sort_scratch_bytes(int64_t capacity);
template <typename PT>
void launch_morton_sort(const ParticleArgs& pa, int ng, double box, int shift, void* sort_scratch,
                        void* particle_scratch, int64_t* block_start, hipStream_t st);

// The deposit after a re-sort into blocks of kBlkCells^3 cells: one
// workgroup per block (launch_block_deposit, particles.hip), usable while the
// particles keep the sorted order and count of block_start.
constexpr int kBlkShift = 4, kBlkCells = 1 << kBlkShift;
inline bool block_deposit_ok(int ng, int sort_shift) {
  return sort_shift == kBlkShift && ng >= 4 * kBlkCells;
}
template <typename PT>
void launch_block_deposit(const ParticleArgs& pa, double drift_coef, int drift, const MeshMap& mm,
                          const int64_t* block_start, uint64_t* counts, uint32_t* flags,
                          hipStream_t st);

// Learned warm start (net.hip).
constexpr int kNetParams = 5 * (27 * 16 * 16 + 16);
constexpr int kNetInputs = 3;   // r0, phi_old, kappa h^2
bool net_size_ok(int n);
void launch_conv(int n, const uint16_t* in, const float* w, const float* bias, int flags,
                 const uint16_t* mask, void* out, hipStream_t st);
size_t wgrad_scratch_bytes(int n);
void launch_conv_wgrad(int n, const uint16_t* in, const uint16_t* g, float* dw, float* db,
                       float* scratch, hipStream_t st);
template <typename RT, typename PT, bool SPLIT>
void launch_net_prep(int n, const RT* r, const PT* phi, float s_r, float s_phi, float kap, const Box* box,
                     uint16_t* act0, hipStream_t st);
void net_forward(int n, const float* params, const uint16_t* act0, uint16_t* a, uint16_t* b,
                 float* out, hipStream_t st);
size_t net_train_scratch_bytes(int n);
void net_train_step(int n, float* params, float* m1, float* m2, int step, float lr,
                    const uint16_t* act0, const float* target, float target_scale, void* scratch,
                    float* loss_out, hipStream_t st);
// mesh.hip helpers for the warm start and for recording solves
template <typename T>
void launch_residual_guess(const double* phi, const float* d, double scale, const double* rhs,
                           T* r_out, int n, const Box& b, double kappa, double* partial,
                           int* nblocks, hipStream_t st);
void launch_apply_guess(double* phi, const float* d, double scale, float* chg, int n,
                        const Box& b, hipStream_t st);
void launch_sum_sq(const double* phi, int n, const Box& b, double* partial, int* nblocks,
                   hipStream_t st);
template <typename T>
void launch_record_start(const T* r_split, const double* phi, int n, const Box& b, float* rec,
                         hipStream_t st);
template <typename T>
void launch_record_accum(const T* e_split, int n, const Box& b, float* dphi, hipStream_t st);

// flags written by kernels
enum : uint32_t { kFlagDomain = 1u, kFlagOverflow = 2u };

// ---------------------------------------------------------------------------
// Per-kernel timing with HIP events (profiler.cpp).  When a context has
// profiling enabled, every launch is bracketed by an event pair on the
// launch stream and charged with its algorithmic bytes; totals are read after
// the next stream synchronisation.
// ---------------------------------------------------------------------------
enum KernelId : int {
  K_FILL, K_DEPOSIT, K_RHS, K_RESIDUAL, K_CORRECT, K_REDUCE, K_SUM_PHI, K_ADD_CONST,
  K_SMOOTH_FIRST, K_SMOOTH, K_RESID_LEVEL, K_RESTRICT, K_PROLONG, K_COARSE,
  K_INTERP_KICK_DRIFT, K_INTERP_FORCE, K_COUNT_KEPT, K_SCAN, K_SCATTER, K_COPY,
  K_SORT, K_GATHER, K_CONV, K_CONV_WGRAD, K_NET_MISC, K_FORCE_MESH, K_LIGHTCONE,
  K_SMOOTH_COARSE, K_ADE, K_FFT, K_FFT_DIVIDE, K_PK, K_SWEEP4, K_SWEEP4_FIRST, K_SWEEP4_COARSE,
  K_SWEEP4_RESID, K_CORRECT_EST, K_RHS_FORCE,
  K_NKERNELS
};
static_assert(K_NKERNELS <= 64, "the profiler's kernel mask holds 64 kernels");
extern const char* const kKernelNames[K_NKERNELS];

struct Profiler {
  bool on = false;
  uint64_t mask = ~0ull;    // kernels bracketed while on (bit = KernelId)
  bool wants(int id) const { return on && ((mask >> id) & 1ull); }
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  std::vector<int> pend_id;
  std::vector<double> pend_bytes;
  std::vector<int> pend_launches;
  double ms[K_NKERNELS] = {};
  double bytes[K_NKERNELS] = {};
  int64_t launches[K_NKERNELS] = {};
  void reset();
  void begin(hipStream_t st);
  // closes the bracket opened by begin: `launches` launches of kernel id,
  // together `bytes` algorithmic bytes
  void end(hipStream_t st, int id, double bytes, int launches = 1);
  void collect();       // call after the stream has been synchronised
  void release();
};

// The profiler of the context making the current call (nullptr: none).
extern thread_local Profiler* g_prof;
inline void prof_begin(hipStream_t st, int id) {
  if (g_prof && g_prof->wants(id)) g_prof->begin(st);
}
inline void prof_end(hipStream_t st, int id, double bytes, int launches = 1) {
  if (g_prof && g_prof->wants(id)) g_prof->end(st, id, bytes, launches);
}

}  // namespace sdpm
