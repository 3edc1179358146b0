// C ABI of libsdpm: context, workspace layout, and the host orchestration of
// one step in the order of the paper's Table 2.  Every numerical operation on
// mesh or particles runs in the HIP kernels of mesh.hip / particles.hip; the
// host computes only FP64 scalars (cosmology.cpp) and the active index box.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>
#include <utility>

#include "internal.h"

using namespace sdpm;

struct sdpm_ctx {
  sdpm_config cfg;
  hipStream_t st = nullptr;
  int nlev_max = 0;      // levels allocated
  int nlev = 0;          // levels in use for the current box
  Level lv[kMaxLevels];
  double* partial = nullptr;
  double* dscal = nullptr;      // reduction outputs
  uint32_t* dflags = nullptr;   // [0] error flags, [1] removed count
  uint64_t* dkept = nullptr;
  uint32_t* bcounts = nullptr;
  uint32_t* boffsets = nullptr;
  void* scratch = nullptr;
  void* sort_scratch = nullptr;
  // first sorted index of each re-sort block (block deposit), valid while
  // the active count is the one it was built for (any positions: particles
  // outside their block's window go to global atomics)
  int64_t* blk_start = nullptr;
  int64_t blk_n = -1;
  float* gmesh = nullptr;       // FP32 force mesh (mixed precision)
  FftPlan fft;                  // periodic FFT solver (SDPM_SOLVER_FFT)
  void* fft_work = nullptr;
  size_t fft_work_bytes = 0;
  // learned warm start
  float* net_params = nullptr;
  uint16_t* net_act0 = nullptr;
  uint16_t* net_a = nullptr;
  uint16_t* net_b = nullptr;
  float* net_out = nullptr;
  void* r_alt = nullptr;
  bool net_ready = false;
  int warm_used = 0;
  // gate of the learned guess (SDPM_WS_LEARNED_GATED), per sub-step kind:
  // moving averages of the guess time and of one V-cycle (with its share of
  // the outer iteration's passes), and the number of solves to skip the net
  // before the next try
  double gate_net_ms = 0.0, gate_cycle_ms = 0.0;
  int gate_skip[2] = {0, 0};
  int gate_backoff[2] = {kGateProbe, kGateProbe};
  // extrapolated start (SDPM_WS_EXTRAP): per solve kind the FP32 change of
  // the last solve (accumulated while it runs) and its conformal step
  float* ex_d[2] = {nullptr, nullptr};
  bool ex_have[2] = {false, false};
  double ex_dtau[2] = {0.0, 0.0};
  double cur_dtau = 0.0;        // conformal step of the sdpm_step in progress (0 otherwise)
  // residual reduction per V-cycle of the last solve of each kind (geometric
  // mean; the two half-step solves differ in kappa and converge at different
  // rates), used to run ahead of the host without a sync per iteration and to
  // pair cycles
  double rho_est[2] = {0.1, 0.1};
  bool rho_measured[2] = {false, false};
  // ||e|| / ||r_old|| of the last outer iteration whose correction pass
  // estimated the residual, per kind of solve (0: not measured yet)
  double e_over_r[2] = {0.0, 0.0};
  // lightcone output
  sdpm_lightcone lc{};
  bool lc_on = false;
  int64_t lc_count = 0;
  // fixed domain (shrink == 0): per-particle "outside at the step's start",
  // the record counter, and the radius at the end of the previous step
  uint8_t* lc_mark = nullptr;
  unsigned long long* lc_counter = nullptr;
  double lc_prev_r = -1.0;
  // solve recording
  float* rec_buf = nullptr;
  int64_t rec_max = 0, rec_count = 0;
  std::vector<double> rec_kappa, rec_rms_r, rec_rms_phi;
  int64_t steps_done = 0;
  double* hpin = nullptr;       // host copies of device scalars
  hipEvent_t ev[12] = {};      // [0..6] step phases, [7] solve-start norms, [8..11] gate timing
  Profiler prof;
  bool bound = false;
  sdpm_particles parts{};
  sdpm_fields fields{};
  int64_t n_active = 0;
  int64_t capacity = 0;
  int periodic = 1;
  Box box{};                    // active box (level 0)
  Box counts_box{};             // cells the last deposit may have written
  char err[512] = {0};
};

namespace {

thread_local char g_create_err[512] = {0};

int fail(sdpm_ctx* c, int code, const char* fmt, ...) {
  char* dst = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, SDPM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
bool same_box(const Box& a, const Box& b) {
  for (int d = 0; d < 3; ++d)
    if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
  return true;
}
int ilog2(int64_t v) {
  int l = 0;
  while ((1ll << l) < v) ++l;
  return l;
}
size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

Box full_box(int n) {
  Box b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = 0;
    b.hi[d] = n - 1;
  }
  return b;
}

bool box_equal(const Box& a, const Box& b) {
  for (int d = 0; d < 3; ++d)
    if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
  return true;
}

int validate(const sdpm_config* c, char* msg, size_t len) {
  if (!c) return snprintf(msg, len, "config is NULL"), SDPM_EINVAL;
  if (!is_pow2(c->ng) || c->ng < 8 || c->ng > 2048)
    return snprintf(msg, len, "ng must be a power of two in [8, 2048] (got %d)", c->ng), SDPM_EINVAL;
  if (c->frac_bits < 1 || c->frac_bits > 16)
    return snprintf(msg, len, "frac_bits must be in [1, 16]"), SDPM_EINVAL;
  if (!(c->box > 0.0) || !std::isfinite(c->box)) return snprintf(msg, len, "box must be > 0"), SDPM_EINVAL;
  if (!(c->omega_m > 0.0) || !(c->c_light > 0.0) || !std::isfinite(c->c_grav))
    return snprintf(msg, len, "omega_m and c_light must be > 0"), SDPM_EINVAL;
  if (c->mg_levels < 2 || c->mg_levels > kMaxLevels)
    return snprintf(msg, len, "mg_levels must be in [2, %d]", kMaxLevels), SDPM_EINVAL;
  const int coarse = c->ng >> (c->mg_levels - 1);
  if (coarse < 4 || coarse > kCoarseMax)
    return snprintf(msg, len, "coarsest multigrid level must have 4..%d cells per axis (ng=%d, levels=%d)",
                    kCoarseMax, c->ng, c->mg_levels), SDPM_EINVAL;
  if (!is_pow2(c->box_align) || c->box_align > c->ng / 4)
    return snprintf(msg, len, "box_align must be a power of two <= ng/4"), SDPM_EINVAL;
  if (c->margin < 2) return snprintf(msg, len, "margin must be >= 2"), SDPM_EINVAL;
  if (c->pre < 1 || c->post < 0 || c->coarse_sweeps < 1 || c->max_outer < 1)
    return snprintf(msg, len, "need pre >= 1, post >= 0, coarse_sweeps >= 1, max_outer >= 1"), SDPM_EINVAL;
  if (!(c->tol > 0.0)) return snprintf(msg, len, "tol must be > 0"), SDPM_EINVAL;
  if (c->precision != SDPM_MIXED && c->precision != SDPM_PLAIN_FP64)
    return snprintf(msg, len, "unknown precision %d", c->precision), SDPM_EINVAL;
  const int ws = c->warm_start & ~SDPM_WS_EXTRAP;
  if (c->warm_start < 0 ||
      (ws != SDPM_WS_PREV && ws != SDPM_WS_LEARNED && ws != SDPM_WS_LEARNED_GATED))
    return snprintf(msg, len, "unknown warm_start %d", c->warm_start), SDPM_EINVAL;
  if (ws != SDPM_WS_PREV && !net_size_ok(c->ng))
    return snprintf(msg, len, "the learned warm start needs ng >= 16"), SDPM_EINVAL;
  if (c->n_initial < 1) return snprintf(msg, len, "n_initial must be >= 1"), SDPM_EINVAL;
  if (c->sort_every < 0 || c->sort_shift < 0 || (c->ng >> c->sort_shift) < 1)
    return snprintf(msg, len, "sort_every and sort_shift must be >= 0, ng >> sort_shift >= 1"), SDPM_EINVAL;
  if (c->solver != SDPM_SOLVER_IMPLICIT && c->solver != SDPM_SOLVER_ADE &&
      c->solver != SDPM_SOLVER_FFT)
    return snprintf(msg, len, "unknown solver %d", c->solver), SDPM_EINVAL;
  if (c->assignment != SDPM_ASSIGN_CIC && c->assignment != SDPM_ASSIGN_TSC)
    return snprintf(msg, len, "unknown assignment %d", c->assignment), SDPM_EINVAL;
  if (c->cycles_per_outer < 1 || c->cycles_per_outer > kMaxCyclesPerOuter)
    return snprintf(msg, len, "cycles_per_outer must be in 1..%d", kMaxCyclesPerOuter), SDPM_EINVAL;
  if (c->solver == SDPM_SOLVER_FFT && c->warm_start != SDPM_WS_PREV)
    return snprintf(msg, len, "the FFT solver takes warm_start SDPM_WS_PREV"), SDPM_EINVAL;
  if (c->solver == SDPM_SOLVER_ADE && (c->c_grav == 0.0 || c->warm_start != SDPM_WS_PREV))
    return snprintf(msg, len, "the ADE solver needs c_grav != 0 and warm_start SDPM_WS_PREV"),
           SDPM_EINVAL;
  return SDPM_OK;
}

size_t mg_elem(const sdpm_config& c) { return c.precision == SDPM_MIXED ? 4 : 8; }
size_t p_elem(const sdpm_config& c) { return c.precision == SDPM_MIXED ? 4 : 8; }

// Workspace layout; with base == nullptr only the size is computed.
size_t carve(const sdpm_config& c, int64_t capacity, char* base, sdpm_ctx* ctx) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const size_t el = mg_elem(c);
  for (int l = 0; l < c.mg_levels; ++l) {
    const int n = c.ng >> l;
    const size_t cells = (size_t)n * n * n;
    char* e = take(cells * el);
    char* r = take(cells * el);
    char* t = take(cells * el);
    char* e_alt = el == 4 && n >= kSweep4Min ? take(cells * el) : nullptr;
    if (ctx) {
      ctx->lv[l].n = n;
      ctx->lv[l].e = e;
      ctx->lv[l].r = r;
      ctx->lv[l].t = t;
      ctx->lv[l].e_alt = e_alt;
      ctx->lv[l].box = full_box(n);
    }
  }
  const Box fb = full_box(c.ng);
  const dim3 g = box_grid(fb);
  const size_t maxblocks = (size_t)g.x * g.y * g.z;
  double* partial = (double*)take(maxblocks * kReduceSlots * sizeof(double));
  double* dscal = (double*)take(64 * sizeof(double));
  uint32_t* dflags = (uint32_t*)take(16 * sizeof(uint32_t));
  uint64_t* dkept = (uint64_t*)take(2 * sizeof(uint64_t));
  unsigned long long* lcc = (unsigned long long*)take(sizeof(unsigned long long));
  uint8_t* lcm = (uint8_t*)take((size_t)capacity);
  const size_t nb = (size_t)((capacity + kChunk - 1) / kChunk) + 1;
  uint32_t* bc = (uint32_t*)take(nb * sizeof(uint32_t));
  uint32_t* bo = (uint32_t*)take(nb * sizeof(uint32_t));
  void* scr = take((size_t)capacity * (3 * sizeof(double) + 3 * p_elem(c) + sizeof(uint32_t)));
  void* sscr = c.sort_every > 0 ? take(sort_scratch_bytes(capacity)) : nullptr;
  int64_t* bst = nullptr;
  if (c.sort_every > 0 && block_deposit_ok(c.ng, c.sort_shift)) {
    const int64_t nb1 = c.ng >> kBlkShift;
    bst = (int64_t*)take((size_t)(nb1 * nb1 * nb1 + 1) * sizeof(int64_t));
  }
  // FP32 force mesh of the mixed-precision step (3 values per cell)
  float* g3 = c.precision == SDPM_MIXED ? (float*)take((size_t)c.ng * c.ng * c.ng * 3 * sizeof(float))
                                        : nullptr;
  if (c.solver == SDPM_SOLVER_FFT) {
    // half spectrum, the transforms' work area (at most the spectrum's size)
    // and the symbol table
    const size_t cb = fft_complex_bytes(c.ng);
    void* cbuf = take(cb);
    void* work = take(cb);
    double* sym = (double*)take((size_t)c.ng * sizeof(double));
    if (ctx) {
      ctx->fft.c = cbuf;
      ctx->fft.sym = sym;
      ctx->fft_work = work;
      ctx->fft_work_bytes = cb;
    }
  }
  if (c.warm_start & SDPM_WS_EXTRAP) {
    const size_t V = (size_t)c.ng * c.ng * c.ng;
    float* d0 = (float*)take(V * sizeof(float));
    float* d1 = (float*)take(V * sizeof(float));
    if (ctx) {
      ctx->ex_d[0] = d0;
      ctx->ex_d[1] = d1;
    }
  }
  if ((c.warm_start & ~SDPM_WS_EXTRAP) != SDPM_WS_PREV) {
    const size_t V = (size_t)c.ng * c.ng * c.ng;
    float* prm = (float*)take(kNetParams * sizeof(float));
    uint16_t* a0 = (uint16_t*)take(V * 16 * sizeof(uint16_t));
    uint16_t* aa = (uint16_t*)take(V * 16 * sizeof(uint16_t));
    uint16_t* ab = (uint16_t*)take(V * 16 * sizeof(uint16_t));
    float* out = (float*)take(V * sizeof(float));
    void* ralt = take(V * mg_elem(c));
    if (ctx) {
      ctx->net_params = prm;
      ctx->net_act0 = a0;
      ctx->net_a = aa;
      ctx->net_b = ab;
      ctx->net_out = out;
      ctx->r_alt = ralt;
    }
  }
  if (ctx) {
    ctx->sort_scratch = sscr;
    ctx->blk_start = bst;
    ctx->gmesh = g3;
    ctx->partial = partial;
    ctx->dscal = dscal;
    ctx->dflags = dflags;
    ctx->dkept = dkept;
    ctx->lc_counter = lcc;
    ctx->lc_mark = lcm;
    ctx->bcounts = bc;
    ctx->boffsets = bo;
    ctx->scratch = scr;
  }
  return off;
}

// Active box for radius r (host; Sec. 2.4 index box, outward rounding).  TSC
// reaches one node further than CIC on each side, so its box takes one more
// cell of margin and keeps the same drift slack between shrinks.
void domain_box(const sdpm_config& c, double r, Box* b, int* periodic) {
  const double h = c.box / c.ng;
  const int64_t A = c.box_align;
  const int m = c.margin + (c.assignment == SDPM_ASSIGN_TSC ? 1 : 0);
  bool fits = true;
  Box out;
  for (int d = 0; d < 3; ++d) {
    int64_t lo = (int64_t)std::floor((c.x_obs[d] - r) / h) - m;
    int64_t hi = (int64_t)std::floor((c.x_obs[d] + r) / h) + m;
    // planes lo-1 and hi+1 on multiples of A (floor / ceil division)
    const int64_t lm = lo - 1, hp = hi + 1;
    const int64_t lf = (lm >= 0 ? lm / A : -((-lm + A - 1) / A)) * A;
    const int64_t hc = (hp >= 0 ? (hp + A - 1) / A : -((-hp) / A)) * A;
    lo = lf + 1;
    hi = hc - 1;
    if (lo < 1 || hi > c.ng - 2) fits = false;
    out.lo[d] = (int)std::max<int64_t>(std::min<int64_t>(lo, c.ng), -1);
    out.hi[d] = (int)std::max<int64_t>(std::min<int64_t>(hi, c.ng), -1);
  }
  if (fits) {
    *b = out;
    *periodic = 0;
  } else {
    *b = full_box(c.ng);
    *periodic = 1;
  }
}

double corner_distance(const sdpm_config& c) {
  double m = 0.0;
  for (int k = 0; k < 8; ++k) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double v = ((k >> d) & 1) ? c.box : 0.0;
      s += (v - c.x_obs[d]) * (v - c.x_obs[d]);
    }
    m = std::max(m, std::sqrt(s));
  }
  return m;
}

// Multigrid level boxes for the current domain.
void set_levels(sdpm_ctx* c) {
  c->lv[0].box = c->periodic ? full_box(c->cfg.ng) : c->box;
  c->nlev = 1;
  for (int l = 1; l < c->nlev_max; ++l) {
    const int n = c->lv[l].n;
    Box b;
    bool empty = false;
    if (c->periodic) {
      b = full_box(n);
    } else {
      const Box& f = c->lv[l - 1].box;
      for (int d = 0; d < 3; ++d) {
        b.lo[d] = (f.lo[d] + 1) >> 1;
        b.hi[d] = std::min(f.hi[d] >> 1, n - 2);
        if (b.hi[d] < b.lo[d]) empty = true;
      }
    }
    if (empty) break;
    c->lv[l].box = b;
    c->nlev = l + 1;
  }
}

// Clears the multigrid correction and scratch arrays (values outside a
// level's box must be zero).
template <typename T>
void clear_levels(sdpm_ctx* c) {
  for (int l = 0; l < c->nlev_max; ++l) {
    const Box fb = full_box(c->lv[l].n);
    launch_fill<T>((T*)c->lv[l].e, c->lv[l].n, fb, (T)0, c->st);
    launch_fill<T>((T*)c->lv[l].t, c->lv[l].n, fb, (T)0, c->st);
    if (c->lv[l].e_alt) launch_fill<T>((T*)c->lv[l].e_alt, c->lv[l].n, fb, (T)0, c->st);
  }
}

void clear_all_levels(sdpm_ctx* c) {
  if (c->cfg.precision == SDPM_MIXED)
    clear_levels<float>(c);
  else
    clear_levels<double>(c);
}

ParticleArgs particle_args(sdpm_ctx* c) {
  ParticleArgs pa;
  for (int d = 0; d < 3; ++d) {
    pa.x[d] = c->parts.x[d];
    pa.p[d] = c->parts.p[d];
  }
  pa.id = c->parts.id;
  pa.n = c->n_active;
  return pa;
}

MeshMap mesh_map(sdpm_ctx* c) {
  MeshMap mm;
  mm.ng = c->cfg.ng;
  mm.frac_bits = c->cfg.frac_bits;
  mm.periodic = c->periodic;
  mm.box = c->cfg.box;
  mm.scale = (double)((int64_t)c->cfg.ng << c->cfg.frac_bits) / c->cfg.box;
  mm.active = c->periodic ? full_box(c->cfg.ng) : c->box;
  mm.tsc = c->cfg.assignment == SDPM_ASSIGN_TSC ? 1 : 0;
  mm.block_shift = c->cfg.sort_shift;
  return mm;
}

int sync_scalars(sdpm_ctx* c, int ndouble) {
  if (ndouble > 0)
    HIP_TRY(c, hipMemcpyAsync(c->hpin, c->dscal, ndouble * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(c, hipMemcpyAsync(c->hpin + 16, c->dflags, 16, hipMemcpyDeviceToHost, c->st));
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  return SDPM_OK;
}

// The conformal step of the sdpm_step in progress, for the extrapolated
// solve start; 0 outside a step.
struct StepDtau {
  sdpm_ctx* c;
  StepDtau(sdpm_ctx* ctx, double dtau) : c(ctx) { c->cur_dtau = dtau; }
  ~StepDtau() { c->cur_dtau = 0.0; }
};

// Makes the context's profiler the current one for the duration of a call.
struct ProfScope {
  explicit ProfScope(sdpm_ctx* c) { g_prof = c ? &c->prof : nullptr; }
  ~ProfScope() { g_prof = nullptr; }
};

// Copies the residual norms of every outer iteration (device slots
// dscal[kNormSlot + it % kNormRing]) to hpin[kHostNorm + ...] and waits.
int sync_norms(sdpm_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->hpin + kHostNorm, c->dscal + kNormSlot, kNormRing * sizeof(double),
                            hipMemcpyDeviceToHost, c->st));
  return sync_scalars(c, 0);
}

// Copies the four sums of the residual estimate (dscal[kEstSlot ..]) to
// hpin[kEstSlot ..] and waits.
int sync_estimate(sdpm_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->hpin + kEstSlot, c->dscal + kEstSlot, 4 * sizeof(double),
                            hipMemcpyDeviceToHost, c->st));
  return sync_scalars(c, 0);
}

// Bound on the distance, in the 2-norm over the box, between the residual
// estimate r_old - A e of launch_correct_est and the FP64 residual
// rhs - A phi of launch_residual after the same correction, from the norms
// of r_old (no), rhs (nb), the new phi (np) and e (ne): r_old carries the
// rounding to T of its FP64 value (at most eps_T / 2 of it per cell); the
// two FP64 residual evaluations, the estimate's own and the FP64 update of
// phi add rounding of at most 9 unit roundoffs of the magnitudes of their
// terms (rhs, r_old, and 12 + kappa times phi or e over the cell and its
// six neighbours, taken as twice the box's norm for the neighbours outside
// a Dirichlet box), bounded here with a factor of 16.
template <typename T>
double estimate_bound(double no, double nb, double np, double ne, double kappa) {
  const double ut = 0.5 * (double)std::numeric_limits<T>::epsilon();
  const double u = 0.5 * std::numeric_limits<double>::epsilon();
  const double g16 = 16.0 * u / (1.0 - 16.0 * u);
  return ut / (1.0 - ut) * no + g16 * (2.0 * nb + no + (12.0 + kappa) * (4.0 * np + 3.0 * ne));
}

uint32_t host_flags(sdpm_ctx* c) { return ((uint32_t*)(c->hpin + 16))[0]; }
uint32_t host_removed(sdpm_ctx* c) { return ((uint32_t*)(c->hpin + 16))[1]; }

int flags_error(sdpm_ctx* c) {
  const uint32_t f = host_flags(c);
  if (f & kFlagOverflow)
    return fail(c, SDPM_EOVERFLOW, "a particle coordinate is not finite");
  if (f & kFlagDomain)
    return fail(c, SDPM_EDOMAIN, "a particle's assignment support (the %s nodes) leaves the active box or the mesh",
                c->cfg.assignment == SDPM_ASSIGN_TSC ? "3^3 TSC" : "2^3 CIC");
  return SDPM_OK;
}

// Extrapolated start (steps only): the solve of kind `slot` starts from
// phi += (dtau / dtau_prev) (change of the same solve kind in the previous
// step); periodic phase only (on the frozen-exterior box the start saved no
// iteration at 512^3).
bool extrap_active(const sdpm_ctx* c, int slot) {
  return slot >= 0 && (c->cfg.warm_start & SDPM_WS_EXTRAP) && c->cur_dtau > 0.0 && c->ex_d[slot] &&
         c->periodic;
}

// rhs = S h^2 (C / (n0/ng^3 2^3B) - ratio) - kappa phi over the box, with
// ratio = n_active / n0 on a periodic mesh (subtracts the exact mean, since
// sum C = n_active 2^3B) and 1 otherwise.  ||rhs||^2 -> dscal[0].  When the
// solve of kind `slot` (-1: none) extrapolates, the same pass applies the
// extrapolated start after reading phi_old for the rhs and starts the running
// change ex_d[slot] that the solve's later updates of phi add to.
//
// With multigrid (mg) and a box wide enough for its vector tiles, the same
// pass also forms the solve's first FP64 residual into level 0's r and its
// norm into dscal[1] (res_ready), and an extrapolated start is left pending
// (pending_scale != 0): phi and the running change are updated by the
// solve's first correction or by launch_apply_start instead, since the
// fused pass reads the neighbours of the cells it would write.
struct RhsOut {
  bool res_ready = false;
  double pending_scale = 0.0;
  bool force_done = false;      // the force mesh of phi was written as well
};
// With g3 (mixed precision, multigrid), the source pass also writes the FP32
// force mesh of phi over the solve's box when it runs as the fused vector
// pass (force_done); the caller takes the force pass otherwise.
RhsOut assemble_rhs(sdpm_ctx* c, double s_source, double kappa, int slot, bool mg = false,
                    float* g3 = nullptr, double inv2h = 0.0) {
  const sdpm_config& g = c->cfg;
  const double h = g.box / g.ng;
  const double nbar = (double)g.n_initial / ((double)g.ng * g.ng * g.ng);
  const double c_scale = s_source * h * h / (nbar * std::ldexp(1.0, 3 * g.frac_bits));
  const double ratio = c->periodic ? (double)c->n_active / (double)g.n_initial : 1.0;
  const double c_off = s_source * h * h * ratio;
  const bool extrap = extrap_active(c, slot);
  const bool apply = extrap && c->ex_have[slot] && c->ex_dtau[slot] > 0.0;
  const double chg_scale = apply ? c->cur_dtau / c->ex_dtau[slot] : 0.0;
  float* chg = extrap ? c->ex_d[slot] : nullptr;
  int nb = 0;
  RhsOut out;
  if (mg) {
    const bool fused =
        g.precision == SDPM_MIXED
            ? launch_rhs_residual<float>(c->fields.counts, c->fields.phi, c->fields.rhs,
                                         (float*)c->lv[0].r, chg, apply, chg_scale, g.ng,
                                         c->lv[0].box, c_scale, c_off, kappa, c->partial, &nb,
                                         c->st, g3, inv2h)
            : launch_rhs_residual<double>(c->fields.counts, c->fields.phi, c->fields.rhs,
                                          (double*)c->lv[0].r, chg, apply, chg_scale, g.ng,
                                          c->lv[0].box, c_scale, c_off, kappa, c->partial, &nb,
                                          c->st);
    if (fused) {
      launch_reduce_final(c->partial, nb, 2, c->dscal, c->st);
      out.res_ready = true;
      out.pending_scale = apply ? chg_scale : 0.0;
      out.force_done = g3 != nullptr && g.precision == SDPM_MIXED;
      return out;
    }
  }
  launch_rhs(c->fields.counts, c->fields.phi, c->fields.rhs, g.ng, c->lv[0].box, c_scale, c_off,
             kappa, chg, chg_scale, apply, c->partial, &nb, c->st);
  launch_reduce_final(c->partial, nb, 1, c->dscal, c->st);
  return out;
}

struct SolveOut {
  double res0 = 0, res = 0, res_guess = 0;
  int iters = 0, vcycles = 0, warm = 0;
};

// FP64 defect correction around V-cycles in T; rhs and ||rhs||^2 (dscal[0])
// must be in place, and with rh.res_ready the first residual and its norm
// (dscal[1]) too.  phi is the initial guess and the result.
template <typename T>
int solve_impl(sdpm_ctx* c, double kappa, int slot, SolveOut* so, RhsOut rh) {
  const sdpm_config& g = c->cfg;
  const Box& b = c->lv[0].box;
  int nb = 0;
  // extrapolated start: applied by assemble_rhs, or pending until the first
  // correction (rh.pending_scale); every later update of phi in this solve
  // is added to the running change chg as well
  const bool extrap = extrap_active(c, slot);
  float* chg = extrap ? c->ex_d[slot] : nullptr;
  double pending = chg ? rh.pending_scale : 0.0;
  auto flush_pending = [&]() {
    if (pending != 0.0) launch_apply_start(c->fields.phi, chg, pending, g.ng, b, c->st);
    pending = 0.0;
  };
  if (!rh.res_ready) {
    launch_residual<T>(c->fields.phi, c->fields.rhs, (T*)c->lv[0].r, g.ng, b, kappa, c->partial,
                       &nb, c->st);
    launch_reduce_final(c->partial, nb, 1, c->dscal + 1, c->st);
  }
  const bool recording = c->rec_buf && c->rec_count < c->rec_max;
  const bool gated = (g.warm_start & ~SDPM_WS_EXTRAP) == SDPM_WS_LEARNED_GATED;
  // The first V-cycle of the first outer iteration does not depend on the
  // norms read next (they decide whether it is used and how many cycles
  // follow it), so when no learned guess or recording can come before it, it
  // is enqueued before the wait and the GPU runs it meanwhile; when the start
  // already meets tol its result is left unused.
  // The copies of the norms go first, the host waits for them alone (event 7).
  const bool spec = !recording && (!c->net_ready || (gated && c->gate_skip[slot] > 0));
  const T* e_spec = nullptr;
  int rc = SDPM_OK;
  if (spec) {
    HIP_TRY(c, hipMemcpyAsync(c->hpin, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipMemcpyAsync(c->hpin + 16, c->dflags, 16, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipEventRecord(c->ev[7], c->st));
    if (gated) HIP_TRY(c, hipEventRecord(c->ev[10], c->st));
    e_spec = vcycle<T>(c->lv, c->nlev, kappa, g.pre, g.post, g.coarse_sweeps, c->periodic != 0,
                       false, c->st);
    HIP_TRY(c, hipEventSynchronize(c->ev[7]));
  } else {
    rc = sync_scalars(c, 2);
    if (rc) return rc;
  }
  const double bn = std::sqrt(c->hpin[0]);
  const double denom = std::max(bn, 1e-300);
  double rn = std::sqrt(c->hpin[1]);
  const double thresh = g.tol * denom;
  so->res0 = rn / denom;
  so->warm = 0;
  const double cells = (double)box_cells(b);
  float* rec = recording ? c->rec_buf + (size_t)c->rec_count * 3 * (size_t)g.ng * g.ng * g.ng : nullptr;
  double rms_phi = 0.0;
  bool try_net = c->net_ready && rn > thresh && rn > 0.0;
  if (try_net && gated && c->gate_skip[slot] > 0) {
    --c->gate_skip[slot];
    try_net = false;
  }
  if (try_net || recording) {
    flush_pending();
    launch_sum_sq(c->fields.phi, g.ng, full_box(g.ng), c->partial, &nb, c->st);
    launch_reduce_final(c->partial, nb, 1, c->dscal + 3, c->st);
    rc = sync_scalars(c, 4);
    if (rc) return rc;
    rms_phi = std::sqrt(c->hpin[3] / ((double)g.ng * g.ng * g.ng));
  }
  if (recording) {
    launch_record_start<T>((const T*)c->lv[0].r, c->fields.phi, g.ng, b, rec, c->st);
    c->rec_kappa.push_back(kappa);
    c->rec_rms_r.push_back(rn / std::sqrt(cells));
    c->rec_rms_phi.push_back(rms_phi);
    ++c->rec_count;
  }
  const double rn_prev = rn;
  bool net_ran = false;
  if (try_net && rms_phi > 0.0) {
    // learned initial guess, kept only if it lowers the residual
    net_ran = true;
    if (gated) HIP_TRY(c, hipEventRecord(c->ev[8], c->st));
    const double rms_r = rn / std::sqrt(cells);
    const Box* pb = c->periodic ? nullptr : &b;
    launch_net_prep<T, double, true>(g.ng, (const T*)c->lv[0].r, c->fields.phi,
                                     (float)(1.0 / rms_r), (float)(1.0 / rms_phi), (float)kappa, pb,
                                     c->net_act0,
                                     c->st);
    net_forward(g.ng, c->net_params, c->net_act0, c->net_a, c->net_b, c->net_out, c->st);
    launch_residual_guess<T>(c->fields.phi, c->net_out, rms_r, c->fields.rhs, (T*)c->r_alt, g.ng, b,
                             kappa, c->partial, &nb, c->st);
    launch_reduce_final(c->partial, nb, 1, c->dscal + 1, c->st);
    if (gated) HIP_TRY(c, hipEventRecord(c->ev[9], c->st));
    rc = sync_scalars(c, 2);
    if (rc) return rc;
    if (gated) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[8], c->ev[9]) == hipSuccess)
        c->gate_net_ms = c->gate_net_ms > 0.0 ? 0.5 * (c->gate_net_ms + ms) : ms;
    }
    const double rg = std::sqrt(c->hpin[1]);
    if (std::isfinite(rg) && rg < rn) {
      launch_apply_guess(c->fields.phi, c->net_out, rms_r, chg, g.ng, b, c->st);
      std::swap(c->lv[0].r, c->r_alt);
      rn = rg;
      so->warm = 1;
    }
  }
  so->res_guess = rn / denom;
  int it = 0, cyc = 0;
  const double rn_start = rn;
  // Outer iterations are enqueued without waiting for their residual norm
  // while the norm predicted from the last known one and the convergence
  // factor per V-cycle of the previous solve stays well above the threshold;
  // then the host waits and reads the norms.  A wrong prediction can only add
  // iterations (the residual keeps falling), never stop early.
  // An outer iteration runs further V-cycles on its defect equation (up to
  // cycles_per_outer) while fewer are predicted to leave the norm above 0.9
  // times the threshold (twice the threshold while the factor per cycle is
  // still a guess): a V-cycle is a linear stationary iteration, so
  // each further cycle reduces the error as a further outer iteration would,
  // down to the rounding floor below, and saves that iteration's FP64
  // correction and residual passes.
  // The cycles of one outer iteration cannot take the defect below the
  // rounding of the correction they store in T: |A de| <= (12 + kappa h^2)
  // (eps_T / 2) |e| with |e| <= |r| / (kappa h^2 + lambda_min), the extreme
  // eigenvalues of the 7-point operator, lambda_min that of the domain's
  // lowest mode (non-constant when periodic; a lower bound, the Dirichlet
  // mode of the box's longest side, otherwise).  The ratio |e| / |r| is
  // taken as measured in the last solve of the same kind where there is one
  // (the estimating correction pass sums both), else at that bound.  Further
  // cycles are added only while their combined factor stays above the floor:
  // at kappa h^2 = 0.113 in FP32 and the bound's ratio (floor 6.4e-6) it
  // allows four cycles of factor above 0.05, for the 512^3 Poisson solve
  // (kappa = 0, floor 4.8e-3) two of factor above 0.07.  Where the floor does
  // stop the residual, the check after the correction finds it and a further
  // outer iteration follows.
  double lam_min;
  {
    const int ext = std::max(b.hi[0] - b.lo[0], std::max(b.hi[1] - b.lo[1], b.hi[2] - b.lo[2])) + 1;
    const double sn = c->periodic ? std::sin(M_PI / g.ng) : std::sin(M_PI / (2.0 * (ext + 1)));
    lam_min = 4.0 * sn * sn;
  }
  const double q_bound = 1.0 / (kappa + lam_min);
  const double q = c->e_over_r[slot] > 0.0 ? std::min(c->e_over_r[slot], q_bound) : q_bound;
  const double floor_rel = 0.5 * (double)std::numeric_limits<T>::epsilon() * (12.0 + kappa) * q;
  double rn_known = rn;
  int it_known = 0, cyc_known = 0;
  while (rn > thresh && it < g.max_outer && std::isfinite(rn)) {
    const bool time_it = gated && it == 0;
    double pred_next = rn_known * std::pow(c->rho_est[slot], cyc - cyc_known + 1);
    double factor = c->rho_est[slot];
    int ncyc = 1;
    const double margin = c->rho_measured[slot] ? kCycleMargin : kCycleMarginGuess;
    while (ncyc < g.cycles_per_outer && pred_next > margin * thresh &&
           factor * c->rho_est[slot] > kFloorMargin * floor_rel) {
      ++ncyc;
      pred_next *= c->rho_est[slot];
      factor *= c->rho_est[slot];
    }
    const bool ahead = it == 0 && e_spec;   // first cycle already enqueued
    if (time_it && !ahead) HIP_TRY(c, hipEventRecord(c->ev[10], c->st));
    const T* e0 = ahead ? e_spec : nullptr;
    for (int q = ahead ? 1 : 0; q < ncyc; ++q)
      e0 = vcycle<T>(c->lv, c->nlev, kappa, g.pre, g.post, g.coarse_sweeps, c->periodic != 0,
                     q > 0, c->st);
    // Where the host waits after this iteration (the test below), the
    // correction pass also estimates the new residual as r_old - A e; when
    // the estimate with its bound is below the threshold, the FP64 residual
    // would be too and its pass is skipped.
    const bool wait = time_it || it + 1 >= g.max_outer || it + 1 - it_known >= kMaxAhead ||
                      !(rn_known * std::pow(c->rho_est[slot], cyc + ncyc - cyc_known) > kAheadMargin * thresh);
    const bool est = wait;
    if (est) {
      launch_correct_est<T>(c->fields.phi, e0, (const T*)c->lv[0].r, chg, pending, kappa, g.ng, b,
                            c->partial, &nb, c->st);
      launch_reduce_final(c->partial, nb, 4, c->dscal + kEstSlot, c->st);
    } else {
      launch_correct<T>(c->fields.phi, e0, chg, pending, g.ng, b, c->st);
    }
    pending = 0.0;
    if (rec) launch_record_accum<T>(e0, g.ng, b, rec + 2 * (size_t)g.ng * g.ng * g.ng, c->st);
    // cost of one V-cycle with its share of the outer iteration's passes
    // (the learned guess's gate weighs the net's cost against it)
    auto cycle_cost = [&]() {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[10], c->ev[11]) == hipSuccess) {
        const double per = ms / ncyc;
        c->gate_cycle_ms = c->gate_cycle_ms > 0.0 ? 0.5 * (c->gate_cycle_ms + per) : per;
      }
    };
    if (time_it && est) HIP_TRY(c, hipEventRecord(c->ev[11], c->st));
    bool met = false;
    if (est) {
      rc = sync_estimate(c);
      if (rc) return rc;
      const double ne = std::sqrt(c->hpin[kEstSlot]);
      const double bound = estimate_bound<T>(std::sqrt(c->hpin[kEstSlot + 1]), bn,
                                             std::sqrt(c->hpin[kEstSlot + 2]),
                                             std::sqrt(c->hpin[kEstSlot + 3]), kappa);
      const double nr = std::sqrt(c->hpin[kEstSlot + 1]), nc = std::sqrt(c->hpin[kEstSlot + 3]);
      if (nr > 0.0 && std::isfinite(nc / nr)) c->e_over_r[slot] = nc / nr;
      if (std::isfinite(ne) && std::isfinite(bound) && (ne + bound) * (1.0 + 1e-9) <= thresh) {
        met = true;
        rn = ne;
      }
    }
    if (!met) {
      launch_residual<T>(c->fields.phi, c->fields.rhs, (T*)c->lv[0].r, g.ng, b, kappa, c->partial,
                         &nb, c->st);
      launch_reduce_final(c->partial, nb, 1, c->dscal + kNormSlot + (it % kNormRing), c->st);
    }
    if (time_it && !est) HIP_TRY(c, hipEventRecord(c->ev[11], c->st));
    ++it;
    cyc += ncyc;
    if (met) {
      if (time_it) cycle_cost();
      break;
    }
    const double pred = rn_known * std::pow(c->rho_est[slot], cyc - cyc_known);
    if (!time_it && it < g.max_outer && it - it_known < kMaxAhead && pred > kAheadMargin * thresh)
      continue;
    rc = sync_norms(c);
    if (rc) return rc;
    if (time_it) cycle_cost();
    rn = std::sqrt(c->hpin[kHostNorm + (it - 1) % kNormRing]);
    rn_known = rn;
    it_known = it;
    cyc_known = cyc;
  }
  flush_pending();      // a start already within tol: no correction took it
  if (cyc > 0 && rn > 0.0 && rn_start > 0.0 && std::isfinite(rn)) {
    const double rho = std::pow(rn / rn_start, 1.0 / cyc);
    if (rho > 0.0 && rho < 1.0) {
      c->rho_est[slot] = std::min(std::max(rho, 1e-3), 0.9);
      c->rho_measured[slot] = true;
    }
  }
  if (gated && net_ran) {
    // V-cycles the guess saved: its residual reduction measured in this
    // solve's own convergence factor per cycle; keep the net for
    // this sub-step kind while that exceeds its cost in iterations, else skip
    // it for a number of solves that doubles with every failed try and scales
    // with how far the net is from paying (cost / saving)
    double saved = 0.0;
    if (so->warm) {
      if (cyc == 0) {
        saved = 1e30;
      } else if (rn > 0.0 && rn_start > 0.0) {
        const double rho = std::pow(rn / rn_start, 1.0 / cyc);
        if (rho > 0.0 && rho < 1.0) saved = std::log(rn_prev / rn_start) / std::log(1.0 / rho);
      }
    }
    const double cost = c->gate_net_ms / std::max(c->gate_cycle_ms, 1e-6);
    if (saved >= cost) {
      c->gate_backoff[slot] = kGateProbe;
      c->gate_skip[slot] = 0;
    } else {
      const double ratio = std::min(cost / std::max(saved, 0.25), (double)kGateProbeMax);
      c->gate_skip[slot] =
          std::min((int)std::ceil(c->gate_backoff[slot] * std::max(ratio, 1.0)), kGateProbeMax);
      c->gate_backoff[slot] = std::min(2 * c->gate_backoff[slot], kGateProbeMax);
    }
  }
  so->iters = it;
  so->vcycles = cyc;
  so->res = rn / denom;
  if (c->periodic && kappa == 0.0) {
    // zero-mean gauge of the singular periodic Poisson problem
    launch_sum_phi(c->fields.phi, g.ng, b, c->partial, &nb, c->st);
    launch_reduce_final(c->partial, nb, 1, c->dscal + 2, c->st);
    rc = sync_scalars(c, 3);
    if (rc) return rc;
    launch_add_const(c->fields.phi, chg, g.ng, b, -c->hpin[2] / (double)box_cells(b), c->st);
  }
  if (extrap) {
    c->ex_have[slot] = true;
    c->ex_dtau[slot] = c->cur_dtau;
  }
  if (!(rn <= thresh))
    return fail(c, SDPM_ENOCONV, "multigrid reached relative residual %.3e > tol %.1e after %d iterations",
                so->res, g.tol, it);
  return SDPM_OK;
}

// Whether the next solve is multigrid (not the FFT of the periodic phase,
// not the ADE sweeps).
bool mg_solve(const sdpm_ctx* c) {
  return c->cfg.solver == SDPM_SOLVER_IMPLICIT || (c->cfg.solver == SDPM_SOLVER_FFT && !c->periodic);
}

int solve(sdpm_ctx* c, double kappa, int slot, SolveOut* so, RhsOut rh = RhsOut{}) {
  if (c->cfg.solver == SDPM_SOLVER_FFT && c->periodic) {
    // exact: no iterations, residual at rounding level (reported as 0)
    *so = SolveOut{};
    const int rc = fft_solve(c->fft, c->fields.rhs, c->fields.phi, kappa, c->st);
    return rc ? fail(c, rc, "hipFFT execution failed") : SDPM_OK;
  }
  return c->cfg.precision == SDPM_MIXED ? solve_impl<float>(c, kappa, slot, so, rh)
                                        : solve_impl<double>(c, kappa, slot, so, rh);
}

int deposit(sdpm_ctx* c, double drift_coef, int drift) {
  launch_fill<uint64_t>(c->fields.counts, c->cfg.ng, c->counts_box, 0ull, c->st);
  c->counts_box = c->periodic ? full_box(c->cfg.ng) : c->box;
  const ParticleArgs pa = particle_args(c);
  const MeshMap mm = mesh_map(c);
  // after a re-sort (and until particles are removed): one workgroup per
  // block with a fixed window; otherwise windows from each workgroup's
  // bounding box
  const bool blocks = c->blk_start && c->blk_n == c->n_active && c->n_active > 0;
  if (blocks) {
    if (c->cfg.precision == SDPM_MIXED)
      launch_block_deposit<float>(pa, drift_coef, drift, mm, c->blk_start, c->fields.counts,
                                  c->dflags, c->st);
    else
      launch_block_deposit<double>(pa, drift_coef, drift, mm, c->blk_start, c->fields.counts,
                                   c->dflags, c->st);
  } else if (c->cfg.precision == SDPM_MIXED) {
    launch_drift_deposit<float>(pa, drift_coef, drift, mm, c->fields.counts, c->dflags, c->st);
  } else {
    launch_drift_deposit<double>(pa, drift_coef, drift, mm, c->fields.counts, c->dflags, c->st);
  }
  return SDPM_OK;
}

// Lightcone radius r: eliminate outside particles (stable partition) and
// update the active box.  `known_removed` < 0: count on the device first.
// Lightcone records of one removal: light = c dtau (0: record at u = 0),
// disp = dtau / a1, a1 the scale factor at the end of the removal, da the step.
struct LcStep {
  double light, disp, a1, da;
};

// Removes the active particles outside radius r (stable partition), records
// them on the lightcone output when lcs != nullptr and it is enabled, and
// updates the active box.  Returns SDPM_EFULL (after all of that) when the
// lightcone output overflowed.
int shrink_impl(sdpm_ctx* c, double r, int64_t known_removed, int64_t* n_removed,
                uint32_t* removed_ids, const LcStep* lcs = nullptr) {
  *n_removed = 0;
  int full = SDPM_OK;
  if (!c->cfg.shrink) return SDPM_OK;
  const int64_t n = c->n_active;
  const double r2 = r * r;
  if (n > 0 && r < corner_distance(c->cfg) * (1.0 + 1e-12) && known_removed != 0) {
    const ParticleArgs pa = particle_args(c);
    // the block deposit's table follows the stable compaction
    const bool blk = c->blk_start && c->blk_n == n;
    const int64_t nb1 = c->cfg.ng >> kBlkShift;
    int64_t* bst = blk ? c->blk_start : nullptr;
    if (c->cfg.precision == SDPM_MIXED)
      launch_compact<float>(pa, c->cfg.x_obs, r2, c->scratch, c->bcounts, c->boffsets, c->dkept,
                            bst, nb1 * nb1 * nb1, c->st);
    else
      launch_compact<double>(pa, c->cfg.x_obs, r2, c->scratch, c->bcounts, c->boffsets, c->dkept,
                             bst, nb1 * nb1 * nb1, c->st);
    HIP_TRY(c, hipMemcpyAsync(c->hpin + 20, c->dkept, sizeof(uint64_t), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    if (c->prof.on) c->prof.collect();
    const int64_t kept = (int64_t)((uint64_t*)(c->hpin + 20))[0];
    *n_removed = n - kept;
    if (removed_ids && *n_removed > 0)
      HIP_TRY(c, hipMemcpyAsync(removed_ids, c->parts.id + kept, *n_removed * sizeof(uint32_t),
                                hipMemcpyDeviceToDevice, c->st));
    if (lcs && c->lc_on && *n_removed > 0) {
      const int64_t room = std::max<int64_t>(c->lc.capacity - c->lc_count, 0);
      const int64_t cnt = std::min(*n_removed, room);
      LcArgs out;
      out.id = c->lc.id;
      out.a = c->lc.a;
      for (int d = 0; d < 3; ++d) {
        out.x[d] = c->lc.x[d];
        out.p[d] = c->lc.p[d];
      }
      if (c->cfg.precision == SDPM_MIXED)
        launch_lightcone<float>(pa, kept, cnt, c->cfg.x_obs, r, lcs->light, lcs->disp, lcs->a1,
                                lcs->da, out, c->lc_count, c->st);
      else
        launch_lightcone<double>(pa, kept, cnt, c->cfg.x_obs, r, lcs->light, lcs->disp, lcs->a1,
                                 lcs->da, out, c->lc_count, c->st);
      c->lc_count += cnt;
      if (cnt < *n_removed) full = SDPM_EFULL;
    }
    c->n_active = kept;
    c->blk_n = blk ? kept : -1;
  }
  Box nb;
  int per = 1;
  domain_box(c->cfg, r, &nb, &per);
  if (!per) {
    if (!c->periodic) {
      for (int d = 0; d < 3; ++d) {
        nb.lo[d] = std::max(nb.lo[d], c->box.lo[d]);
        nb.hi[d] = std::min(nb.hi[d], c->box.hi[d]);
      }
    }
    if (c->periodic || !box_equal(nb, c->box)) {
      c->periodic = 0;
      c->box = nb;
      set_levels(c);
      clear_all_levels(c);
    }
  }
  if (full) return fail(c, SDPM_EFULL, "lightcone output full at %lld records; later records dropped",
                        (long long)c->lc_count);
  return SDPM_OK;
}

void sort_particles(sdpm_ctx* c) {
  if (!c->sort_scratch || c->n_active <= 1) return;
  const ParticleArgs pa = particle_args(c);
  if (c->cfg.precision == SDPM_MIXED)
    launch_morton_sort<float>(pa, c->cfg.ng, c->cfg.box, c->cfg.sort_shift, c->sort_scratch,
                              c->scratch, c->blk_start, c->st);
  else
    launch_morton_sort<double>(pa, c->cfg.ng, c->cfg.box, c->cfg.sort_shift, c->sort_scratch,
                               c->scratch, c->blk_start, c->st);
  c->blk_n = c->blk_start ? c->n_active : -1;
}

void fill_state(sdpm_ctx* c, sdpm_step_stats* o) {
  o->n_active = c->n_active;
  for (int d = 0; d < 3; ++d) {
    o->lo[d] = c->periodic ? 0 : c->box.lo[d];
    o->hi[d] = c->periodic ? c->cfg.ng - 1 : c->box.hi[d];
  }
  o->periodic = c->periodic;
}

int check_ready(sdpm_ctx* c) {
  if (!c) return SDPM_EINVAL;
  if (!c->bound) return fail(c, SDPM_ESTATE, "no particles/fields bound (call sdpm_bind first)");
  return SDPM_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int sdpm_config_default(sdpm_config* cfg, int32_t ng, double box) {
  if (!cfg) return SDPM_EINVAL;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->ng = ng;
  cfg->frac_bits = 14;
  cfg->box = box;
  cfg->omega_m = 0.3;
  cfg->omega_l = 0.7;
  cfg->c_light = 2997.92458;
  cfg->c_grav = 0.0;
  for (int d = 0; d < 3; ++d) cfg->x_obs[d] = 0.5 * box;
  cfg->shrink = 0;
  cfg->margin = 2;
  int lv = 6;
  if (is_pow2(ng) && ng >= 8) {
    const int lg = ilog2(ng);
    lv = std::max(2, std::min(lg - 3, kMaxLevels));   // coarsest 16 cells (8 or 4 if ng < 32)
    if ((ng >> (lv - 1)) < 4) lv = 2;
  }
  cfg->mg_levels = lv;
  cfg->box_align = 1 << (lv - 1);
  cfg->pre = 2;
  cfg->post = 2;
  cfg->coarse_sweeps = 64;
  cfg->max_outer = 50;
  cfg->tol = 1e-8;
  cfg->precision = SDPM_MIXED;
  cfg->warm_start = SDPM_WS_PREV;
  cfg->n_initial = (int64_t)ng * ng * ng;
  cfg->sort_every = 0;
  cfg->sort_shift = ng >= 64 ? 4 : 0;   // Morton order of 16^3-cell blocks
  cfg->solver = SDPM_SOLVER_IMPLICIT;
  cfg->cycles_per_outer = 4;
  cfg->assignment = SDPM_ASSIGN_CIC;
  return SDPM_OK;
}

int sdpm_step_scalars(const sdpm_config* cfg, double a, double da, double out[7]) {
  char msg[256];
  const int rc = validate(cfg, msg, sizeof msg);
  if (rc) return fail(nullptr, rc, "%s", msg);
  if (!out || !(a > 0.0) || !(da > 0.0)) return fail(nullptr, SDPM_EINVAL, "need a > 0, da > 0");
  const StepScalars s = step_scalars(*cfg, a, da);
  out[0] = s.dtau;
  out[1] = s.a_half;
  out[2] = s.s_half;
  out[3] = s.kappa1_h2;
  out[4] = s.kappa2_h2;
  out[5] = s.r_lc_end;
  out[6] = s.c_g;
  return SDPM_OK;
}

int sdpm_lightcone_radius(const sdpm_config* cfg, double a, double* r) {
  if (!cfg || !r || !(a > 0.0)) return SDPM_EINVAL;
  *r = lightcone_radius(a, cfg->omega_m, cfg->omega_l, cfg->c_light);
  return SDPM_OK;
}

int sdpm_domain_box(const sdpm_config* cfg, double r, int32_t lo[3], int32_t hi[3],
                    int32_t* periodic) {
  char msg[256];
  const int rc = validate(cfg, msg, sizeof msg);
  if (rc) return fail(nullptr, rc, "%s", msg);
  if (!lo || !hi || !periodic || !(r >= 0.0)) return SDPM_EINVAL;
  Box b;
  int per;
  domain_box(*cfg, r, &b, &per);
  for (int d = 0; d < 3; ++d) {
    lo[d] = b.lo[d];
    hi[d] = b.hi[d];
  }
  *periodic = per;
  return SDPM_OK;
}

int sdpm_workspace_bytes(const sdpm_config* cfg, int64_t capacity, int64_t* bytes) {
  char msg[256];
  const int rc = validate(cfg, msg, sizeof msg);
  if (rc) return fail(nullptr, rc, "%s", msg);
  if (!bytes || capacity < 0 || capacity >= (1ll << 32))
    return fail(nullptr, SDPM_EINVAL, "capacity must be in [0, 2^32)");
  *bytes = (int64_t)carve(*cfg, capacity, nullptr, nullptr);
  return SDPM_OK;
}

int sdpm_create(const sdpm_config* cfg, void* workspace, int64_t ws_bytes, void* hip_stream,
                sdpm_ctx** out) {
  char msg[256];
  int rc = validate(cfg, msg, sizeof msg);
  if (rc) return fail(nullptr, rc, "%s", msg);
  if (!out || !workspace) return fail(nullptr, SDPM_EINVAL, "out and workspace must be non-NULL");
  sdpm_ctx* c = new (std::nothrow) sdpm_ctx;
  if (!c) return fail(nullptr, SDPM_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->st = (hipStream_t)hip_stream;
  // largest particle capacity whose layout fits the workspace
  const size_t fixed = carve(*cfg, 0, nullptr, nullptr);
  if ((size_t)ws_bytes < fixed) {
    delete c;
    return fail(nullptr, SDPM_ENOMEM, "workspace of %lld bytes < %zu required",
                (long long)ws_bytes, fixed);
  }
  const size_t per = 3 * sizeof(double) + 3 * p_elem(*cfg) + sizeof(uint32_t);
  int64_t lo = 0, hi = (int64_t)(((size_t)ws_bytes - fixed) / per) + 1;
  hi = std::min<int64_t>(hi, (1ll << 32) - 1);
  while (lo < hi) {  // invariant: carve(lo) fits
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (carve(*cfg, mid, nullptr, nullptr) <= (size_t)ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t cap = lo;
  c->capacity = cap;
  carve(*cfg, cap, (char*)workspace, c);
  c->nlev_max = cfg->mg_levels;
  c->periodic = 1;
  c->box = full_box(cfg->ng);
  c->counts_box = full_box(cfg->ng);
  set_levels(c);
  // pinned, so that the scalar copies to the host are asynchronous (into
  // pageable memory the runtime returns from each copy only once it is done)
  if (hipHostMalloc((void**)&c->hpin, kHostScalars * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      !c->hpin) {
    c->hpin = nullptr;
    delete c;
    return fail(nullptr, SDPM_ENOMEM, "pinned host allocation failed");
  }
  std::memset(c->hpin, 0, kHostScalars * sizeof(double));
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipHostFree(c->hpin);
      delete c;
      return fail(nullptr, SDPM_EHIP, "hipEventCreate failed");
    }
  }
  clear_all_levels(c);
  if (cfg->solver == SDPM_SOLVER_FFT) {
    char msg[256];
    const int frc = fft_init(&c->fft, cfg->ng, c->fft.c, c->fft_work, c->fft_work_bytes, c->fft.sym,
                             c->st, msg, sizeof msg);
    if (frc) {
      fft_destroy(&c->fft);
      for (auto& e : c->ev) (void)hipEventDestroy(e);
      (void)hipHostFree(c->hpin);
      delete c;
      return fail(nullptr, frc, "%s", msg);
    }
  }
  *out = c;
  return SDPM_OK;
}

int sdpm_bind(sdpm_ctx* c, const sdpm_particles* parts, const sdpm_fields* fields,
              int64_t n_active) {
  ProfScope prof_scope(c);
  if (!c) return SDPM_EINVAL;
  if (!parts || !fields || !fields->phi || !fields->rhs || !fields->counts)
    return fail(c, SDPM_EINVAL, "particles and fields must be non-NULL");
  if (n_active < 0 || n_active > parts->capacity)
    return fail(c, SDPM_EINVAL, "n_active must be in [0, capacity]");
  if (parts->capacity > c->capacity)
    return fail(c, SDPM_ENOMEM, "particle capacity %lld exceeds what the workspace holds (%lld)",
                (long long)parts->capacity, (long long)c->capacity);
  if (n_active > 0)
    for (int d = 0; d < 3; ++d)
      if (!parts->x[d] || !parts->p[d] || !parts->id)
        return fail(c, SDPM_EINVAL, "particle arrays must be non-NULL");
  c->parts = *parts;
  c->fields = *fields;
  c->n_active = n_active;
  c->blk_n = -1;
  c->periodic = 1;
  c->box = full_box(c->cfg.ng);
  c->counts_box = full_box(c->cfg.ng);
  set_levels(c);
  clear_all_levels(c);
  HIP_TRY(c, hipMemsetAsync(c->dflags, 0, 16 * sizeof(uint32_t), c->st));
  c->bound = true;
  c->steps_done = 0;
  c->err[0] = 0;
  return SDPM_OK;
}

int sdpm_init_potential(sdpm_ctx* c, double a, sdpm_step_stats* out) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(a > 0.0) || a > 1.0) return fail(c, SDPM_EINVAL, "a must be in (0, 1]");
  sdpm_step_stats st{};
  int64_t removed = 0;
  const double r = lightcone_radius(a, c->cfg.omega_m, c->cfg.omega_l, c->cfg.c_light);
  const LcStep at_a{0.0, 0.0, a, 0.0};
  rc = shrink_impl(c, r, -1, &removed, nullptr, &at_a);
  const int full = rc == SDPM_EFULL ? rc : SDPM_OK;
  c->lc_prev_r = r;   // the first step's start radius (fixed-domain lightcone)
  if (rc && !full) return rc;
  HIP_TRY(c, hipMemsetAsync(c->dflags, 0, 16 * sizeof(uint32_t), c->st));
  launch_fill<uint64_t>(c->fields.counts, c->cfg.ng, full_box(c->cfg.ng), 0ull, c->st);
  deposit(c, 0.0, 0);
  const RhsOut rh = assemble_rhs(c, 1.5 * c->cfg.omega_m / a, 0.0, 0, mg_solve(c));
  SolveOut so;
  const int src = solve(c, 0.0, 0, &so, rh);
  rc = flags_error(c);
  st.n_removed = removed;
  st.outer_iters[0] = so.iters;
  st.vcycles = so.vcycles;
  st.res0[0] = so.res0;
  st.res[0] = so.res;
  st.r_lc = r;
  fill_state(c, &st);
  if (out) *out = st;
  if (rc) return rc;
  return src ? src : full;
}

int sdpm_step(sdpm_ctx* c, double a, double da, sdpm_step_stats* out) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(a > 0.0) || !(da > 0.0) || a + da > 1.0 + 1e-12)
    return fail(c, SDPM_EINVAL, "need a > 0, da > 0 and a + da <= 1");
  const sdpm_config& g = c->cfg;
  const StepScalars sc = step_scalars(g, a, da);
  const double h = g.box / g.ng;
  sdpm_step_stats st{};
  st.dtau = sc.dtau;
  st.a_half = sc.a_half;
  st.kappa_h2[0] = sc.kappa1_h2;
  st.kappa_h2[1] = sc.kappa2_h2;
  st.r_lc = sc.r_lc_end;
  HIP_TRY(c, hipMemsetAsync(c->dflags, 0, 16 * sizeof(uint32_t), c->st));
  HIP_TRY(c, hipEventRecord(c->ev[0], c->st));
  if (g.sort_every > 0 && c->steps_done % g.sort_every == 0) sort_particles(c);
  ++c->steps_done;
  // lightcone output on a fixed domain: who is outside at the step's start
  // (the radius at the end of the previous step, or at a for the first)
  const bool lc_fixed = !g.shrink && c->lc_on && c->n_active > 0;
  if (lc_fixed) {
    const double r0 = c->lc_prev_r > 0.0 ? c->lc_prev_r
                                          : lightcone_radius(a, g.omega_m, g.omega_l, g.c_light);
    launch_lc_mark(particle_args(c), g.x_obs, r0 * r0, c->lc_mark, c->st);
  }
  // drift dtau/2 with a(t), then density at t + dt/2   (Table 2 rows 1-2);
  // the deposit does not store the drifted positions, the interpolation pass
  // recomputes them: an error before it leaves the particles untouched
  deposit(c, 0.5 * sc.dtau / a, 1);
  HIP_TRY(c, hipEventRecord(c->ev[1], c->st));
  // Phi from t to t + dt/2                              (row 3)
  const bool ade = g.solver == SDPM_SOLVER_ADE;
  const StepDtau step_dtau(c, sc.dtau);
  const RhsOut rh1 = assemble_rhs(c, sc.s_half, ade ? 0.0 : sc.kappa1_h2, 0, !ade && mg_solve(c));
  HIP_TRY(c, hipEventRecord(c->ev[2], c->st));
  SolveOut s1;
  int src1 = SDPM_OK;
  if (ade) {
    // the paper's ADE: a forward sweep with the mid-step source f = rhs
    launch_ade_sweep(c->fields.phi, c->fields.rhs, g.ng, c->lv[0].box, c->periodic != 0,
                     1.0 / sc.kappa1_h2, true, c->st);
  } else {
    src1 = solve(c, sc.kappa1_h2, 0, &s1, rh1);
    if (src1 && src1 != SDPM_ENOCONV) return src1;
  }
  HIP_TRY(c, hipEventRecord(c->ev[3], c->st));
  // The second half sub-step's source pass (row 7: the same density and the
  // potential just solved for) does not depend on the particle pass; when
  // its box is the force mesh's, it runs first and writes the force mesh too.
  RhsOut rh2;
  bool rh2_done = false;
  if (!ade && sc.kappa2_h2 > 0.0 && g.precision == SDPM_MIXED && mg_solve(c) &&
      same_box(mesh_map(c).active, c->lv[0].box)) {
    rh2 = assemble_rhs(c, sc.s_half, sc.kappa2_h2, 1, true, c->gmesh, 0.5 / h);
    rh2_done = true;
  }
  // grad Phi, CIC interpolation, kick with a(t+dt/2), drift with a(t+dt)  (rows 4-6)
  const bool removal = g.shrink && c->n_active > 0 &&
                       sc.r_lc_end < corner_distance(g) * (1.0 + 1e-12);
  {
    const ParticleArgs pa = particle_args(c);
    const MeshMap mm = mesh_map(c);
    // the first drift is applied here (the deposit only used it)
    const double drift0 = 0.5 * sc.dtau / a;
    const double kick = sc.a_half * sc.dtau, drift = 0.5 * sc.dtau / (a + da);
    if (g.precision == SDPM_MIXED) {
      // FP32 force mesh (FP64 differences), then 12-byte gathers per CIC cell
      if (!rh2.force_done) launch_force_mesh(c->fields.phi, c->gmesh, g.ng, mm.active, 0.5 / h, c->st);
      launch_interp_kick_drift<float>(pa, c->fields.phi, c->gmesh, mm, 0.5 / h, drift0, kick, drift,
                                      g.x_obs, sc.r_lc_end * sc.r_lc_end, removal, c->dflags + 1,
                                      c->dflags, c->st);
    } else {
      launch_interp_kick_drift<double>(pa, c->fields.phi, nullptr, mm, 0.5 / h, drift0, kick,
                                       drift, g.x_obs, sc.r_lc_end * sc.r_lc_end, removal,
                                       c->dflags + 1, c->dflags, c->st);
    }
  }
  HIP_TRY(c, hipEventRecord(c->ev[4], c->st));
  // Phi from t + dt/2 to t + dt with the same density    (row 7)
  SolveOut s2;
  int src2 = SDPM_OK;
  // a multigrid solve waits for the GPU at least once, after the particle
  // pass above: the flags and the removal count it copied to the host are
  // then already those of this step
  bool flags_read = false;
  if (ade) {
    // the same source, the sweep in the other direction
    launch_ade_sweep(c->fields.phi, c->fields.rhs, g.ng, c->lv[0].box, c->periodic != 0,
                     1.0 / sc.kappa2_h2, false, c->st);
  } else if (sc.kappa2_h2 > 0.0) {
    const bool mg = mg_solve(c);
    if (!rh2_done) rh2 = assemble_rhs(c, sc.s_half, sc.kappa2_h2, 1, mg);
    src2 = solve(c, sc.kappa2_h2, 1, &s2, rh2);
    if (src2 && src2 != SDPM_ENOCONV) return src2;
    flags_read = mg;
  }
  HIP_TRY(c, hipEventRecord(c->ev[5], c->st));
  if (lc_fixed) {
    // record the particles that crossed the lightcone during the step
    HIP_TRY(c, hipMemsetAsync(c->lc_counter, 0, sizeof(unsigned long long), c->st));
    LcArgs out;
    out.id = c->lc.id;
    out.a = c->lc.a;
    for (int d = 0; d < 3; ++d) {
      out.x[d] = c->lc.x[d];
      out.p[d] = c->lc.p[d];
    }
    const double r1 = sc.r_lc_end;
    if (g.precision == SDPM_MIXED)
      launch_lc_cross<float>(particle_args(c), g.x_obs, r1 * r1, r1, g.c_light * sc.dtau,
                             sc.dtau / (a + da), a + da, da, c->lc_mark, out, c->lc_count,
                             c->lc.capacity, c->lc_counter, c->st);
    else
      launch_lc_cross<double>(particle_args(c), g.x_obs, r1 * r1, r1, g.c_light * sc.dtau,
                              sc.dtau / (a + da), a + da, da, c->lc_mark, out, c->lc_count,
                              c->lc.capacity, c->lc_counter, c->st);
    HIP_TRY(c, hipMemcpyAsync(c->hpin + kHostLcCount, c->lc_counter, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->st));
  }
  c->lc_prev_r = sc.r_lc_end;
  if (lc_fixed || !flags_read) {
    rc = sync_scalars(c, 1);
    if (rc) return rc;
  }
  int lc_full = SDPM_OK;
  if (lc_fixed) {
    const int64_t crossed = (int64_t)((const unsigned long long*)(c->hpin + kHostLcCount))[0];
    if (c->lc_count + crossed > c->lc.capacity) lc_full = SDPM_EFULL;
    c->lc_count = std::min(c->lc_count + crossed, (int64_t)c->lc.capacity);
  }
  const int ferr = flags_error(c);
  // lightcone at t + dt: eliminate particles and cells  (last row)
  int64_t removed = 0;
  int full = SDPM_OK;
  if (!ferr) {
    const LcStep lcs{g.c_light * sc.dtau, sc.dtau / (a + da), a + da, da};
    rc = shrink_impl(c, sc.r_lc_end, removal ? (int64_t)host_removed(c) : 0, &removed, nullptr,
                     &lcs);
    if (rc == SDPM_EFULL)
      full = rc;
    else if (rc)
      return rc;
  }
  HIP_TRY(c, hipEventRecord(c->ev[6], c->st));
  HIP_TRY(c, hipEventSynchronize(c->ev[6]));
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  const int pairs[7][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {5, 6}, {0, 6}};
  for (int q = 0; q < 7; ++q) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[pairs[q][0]], c->ev[pairs[q][1]]);
    st.ms[q] = ms;
  }
  // solve 1 includes rhs assembly in ms[2]; report rhs separately as ms[1]
  st.n_removed = removed;
  st.outer_iters[0] = s1.iters;
  st.outer_iters[1] = s2.iters;
  st.vcycles = s1.vcycles + s2.vcycles;
  st.warm_used = s1.warm + s2.warm;
  st.res0[0] = s1.res0;
  st.res[0] = s1.res;
  st.res0[1] = s2.res0;
  st.res[1] = s2.res;
  st.res_guess[0] = s1.res_guess;
  st.res_guess[1] = s2.res_guess;
  fill_state(c, &st);
  if (out) *out = st;
  if (ferr) return ferr;
  if (src1) return src1;
  if (src2) return src2;
  return full ? full : lc_full;
}

int sdpm_shrink_radius(sdpm_ctx* c, double r, int64_t* n_removed, uint32_t* removed_ids_dev) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(r >= 0.0)) return fail(c, SDPM_EINVAL, "radius must be >= 0");
  int64_t nr = 0;
  rc = shrink_impl(c, r, -1, &nr, removed_ids_dev);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  if (n_removed) *n_removed = nr;
  return SDPM_OK;
}

int sdpm_shrink(sdpm_ctx* c, double a, int64_t* n_removed, uint32_t* removed_ids_dev) {
  if (!c) return SDPM_EINVAL;
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(a > 0.0) || a > 1.0) return fail(c, SDPM_EINVAL, "a must be in (0, 1]");
  int64_t nr = 0;
  const LcStep at_a{0.0, 0.0, a, 0.0};
  rc = shrink_impl(c, lightcone_radius(a, c->cfg.omega_m, c->cfg.omega_l, c->cfg.c_light), -1, &nr,
                   removed_ids_dev, &at_a);
  if (rc && rc != SDPM_EFULL) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  if (n_removed) *n_removed = nr;
  return rc;
}

int sdpm_set_lightcone(sdpm_ctx* c, const sdpm_lightcone* out) {
  if (!c) return SDPM_EINVAL;
  if (!out) {
    c->lc_on = false;
    c->lc = sdpm_lightcone{};
    c->lc_count = 0;
    return SDPM_OK;
  }
  if (out->capacity < 0 || (out->capacity > 0 && (!out->id || !out->a || !out->x[0] || !out->x[1] ||
                                                  !out->x[2] || !out->p[0] || !out->p[1] ||
                                                  !out->p[2])))
    return fail(c, SDPM_EINVAL, "lightcone output: null array or negative capacity");
  c->lc = *out;
  c->lc_on = true;
  c->lc_count = 0;
  return SDPM_OK;
}

int sdpm_lightcone_count(sdpm_ctx* c, int64_t* count) {
  if (!c || !count) return SDPM_EINVAL;
  *count = c->lc_count;
  return SDPM_OK;
}

int sdpm_get_state(sdpm_ctx* c, sdpm_step_stats* out) {
  if (!c || !out) return SDPM_EINVAL;
  std::memset(out, 0, sizeof(*out));
  fill_state(c, out);
  return SDPM_OK;
}

int sdpm_deposit(sdpm_ctx* c) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemsetAsync(c->dflags, 0, 16 * sizeof(uint32_t), c->st));
  deposit(c, 0.0, 0);
  rc = sync_scalars(c, 0);
  if (rc) return rc;
  return flags_error(c);
}

int sdpm_solve(sdpm_ctx* c, double kappa_h2, double s_source, sdpm_step_stats* out) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(kappa_h2 >= 0.0) || !std::isfinite(s_source))
    return fail(c, SDPM_EINVAL, "kappa_h2 must be >= 0 and s finite");
  const RhsOut rh = assemble_rhs(c, s_source, kappa_h2, 0, mg_solve(c));
  SolveOut so;
  rc = solve(c, kappa_h2, 0, &so, rh);
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->outer_iters[0] = so.iters;
    out->vcycles = so.vcycles;
    out->warm_used = so.warm;
    out->res0[0] = so.res0;
    out->res[0] = so.res;
    out->res_guess[0] = so.res_guess;
    out->kappa_h2[0] = kappa_h2;
    fill_state(c, out);
  }
  return rc;
}

int sdpm_ade_sweep(sdpm_ctx* c, double lam, int forward) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!(lam > 0.0) || !std::isfinite(lam))
    return fail(c, SDPM_EINVAL, "lam must be finite and > 0");
  launch_ade_sweep(c->fields.phi, c->fields.rhs, c->cfg.ng, c->lv[0].box, c->periodic != 0, lam,
                   forward != 0, c->st);
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  return SDPM_OK;
}

int sdpm_sort(sdpm_ctx* c) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!c->sort_scratch)
    return fail(c, SDPM_ESTATE, "the context was created with sort_every = 0 (no sort workspace)");
  sort_particles(c);
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  return SDPM_OK;
}

int sdpm_interp_force(sdpm_ctx* c, double* g_dev[3]) {
  ProfScope prof_scope(c);
  int rc = check_ready(c);
  if (rc) return rc;
  if (!g_dev || (c->n_active > 0 && (!g_dev[0] || !g_dev[1] || !g_dev[2])))
    return fail(c, SDPM_EINVAL, "g_dev arrays must be non-NULL");
  HIP_TRY(c, hipMemsetAsync(c->dflags, 0, 16 * sizeof(uint32_t), c->st));
  const double h = c->cfg.box / c->cfg.ng;
  launch_interp_force(particle_args(c), c->fields.phi, mesh_map(c), 0.5 / h,
                      c->n_active ? g_dev[0] : nullptr, c->n_active ? g_dev[1] : nullptr,
                      c->n_active ? g_dev[2] : nullptr, c->dflags, c->st);
  rc = sync_scalars(c, 0);
  if (rc) return rc;
  return flags_error(c);
}

int sdpm_set_warmstart_weights(sdpm_ctx* c, const float* params_host, int64_t n_params) {
  if (!c) return SDPM_EINVAL;
  if (!c->net_params)
    return fail(c, SDPM_ESTATE, "the context was created with warm_start = SDPM_WS_PREV");
  if (!params_host || n_params != kNetParams)
    return fail(c, SDPM_EINVAL, "expected %d parameters", kNetParams);
  HIP_TRY(c, hipMemcpyAsync(c->net_params, params_host, kNetParams * sizeof(float),
                            hipMemcpyHostToDevice, c->st));
  HIP_TRY(c, hipStreamSynchronize(c->st));
  c->net_ready = true;
  return SDPM_OK;
}

int sdpm_record(sdpm_ctx* c, float* buf_dev, int64_t max_solves) {
  if (!c) return SDPM_EINVAL;
  if (max_solves < 0 || (max_solves > 0 && !buf_dev)) return fail(c, SDPM_EINVAL, "bad record buffer");
  if (c->net_ready) return fail(c, SDPM_ESTATE, "recording needs the plain warm start");
  c->rec_buf = max_solves ? buf_dev : nullptr;
  c->rec_max = max_solves;
  c->rec_count = 0;
  c->rec_kappa.clear();
  c->rec_rms_r.clear();
  c->rec_rms_phi.clear();
  return SDPM_OK;
}

int sdpm_record_info(sdpm_ctx* c, int64_t* count, double* kappa_h2, double* rms_r,
                     double* rms_phi, int64_t max) {
  if (!c || !count) return SDPM_EINVAL;
  *count = c->rec_count;
  for (int64_t q = 0; q < c->rec_count && q < max; ++q) {
    if (kappa_h2) kappa_h2[q] = c->rec_kappa[q];
    if (rms_r) rms_r[q] = c->rec_rms_r[q];
    if (rms_phi) rms_phi[q] = c->rec_rms_phi[q];
  }
  return SDPM_OK;
}

int sdpm_conv3d(int32_t n, const void* in_bf16, const float* w, const float* bias, int32_t flags,
                const void* mask_bf16, void* out, void* stream) {
  if (!net_size_ok(n) || !in_bf16 || !w || !out)
    return fail(nullptr, SDPM_EINVAL, "conv3d: n must be a power of two >= 16, pointers non-NULL");
  if (flags != 0 && flags != SDPM_CONV_RELU && flags != SDPM_CONV_OUT_FP32_CH0 &&
      flags != SDPM_CONV_BACKWARD_DATA &&
      flags != (SDPM_CONV_BACKWARD_DATA | SDPM_CONV_MASK))
    return fail(nullptr, SDPM_EINVAL, "conv3d: unsupported flag combination %d", flags);
  if ((flags & SDPM_CONV_MASK) && !mask_bf16) return fail(nullptr, SDPM_EINVAL, "conv3d: mask is NULL");
  launch_conv(n, (const uint16_t*)in_bf16, w, bias, flags, (const uint16_t*)mask_bf16, out,
              (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "conv3d launch failed");
}

int sdpm_rb_sweeps(int32_t n, const float* e, float* e_out, const float* r, float scale,
                   float inv_diag, int32_t first, int32_t fused, float* t_out, float kappa_h2,
                   const int32_t* box, void* stream) {
  if (n < 64 || n > 2048 || (n & (n - 1)) || !e_out || !r || (!first && !e))
    return fail(nullptr, SDPM_EINVAL, "rb_sweeps: n a power of two in [64, 2048], pointers non-NULL");
  if (fused && !first && e == e_out)
    return fail(nullptr, SDPM_EINVAL, "rb_sweeps: the fused form needs e_out != e");
  if (t_out && (!(scale > 0.0f) || t_out == e_out || t_out == e || t_out == r))
    return fail(nullptr, SDPM_EINVAL, "rb_sweeps: t_out needs scale > 0 and its own array");
  Box b{};
  if (box) {
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = box[d];
      b.hi[d] = box[3 + d];
      if (b.lo[d] < 1 || b.hi[d] > n - 2 || b.hi[d] < b.lo[d])
        return fail(nullptr, SDPM_EINVAL, "rb_sweeps: the box must keep a plane from every face");
    }
  }
  launch_sweeps4(e, e_out, r, n, scale, inv_diag, first != 0, fused != 0, t_out,
                 t_out ? 1.0f / scale : 0.0f, kappa_h2, box ? &b : nullptr, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "rb_sweeps launch failed");
}

int sdpm_pk_workspace_bytes(int32_t ng, int64_t* bytes) {
  if (ng < 8 || ng > 1024 || (ng & (ng - 1)) || !bytes)
    return fail(nullptr, SDPM_EINVAL, "ng must be a power of two in [8, 1024]");
  *bytes = (int64_t)pk_workspace_bytes(ng);
  return SDPM_OK;
}

int sdpm_power_spectrum(const double* const x_dev[3], int64_t n, double box, int32_t ng,
                        int32_t flags, void* workspace, int64_t ws_bytes, void* hip_stream,
                        double* k, double* p, double* p_raw, int64_t* modes) {
  if (ng < 8 || ng > 1024 || (ng & (ng - 1)) || n <= 0 || !(box > 0.0) || !std::isfinite(box) ||
      !x_dev || !x_dev[0] || !x_dev[1] || !x_dev[2] || !workspace || !k || !p || !modes ||
      (flags & ~(SDPM_PK_SHOT | SDPM_PK_JING)))
    return fail(nullptr, SDPM_EINVAL,
                "power_spectrum: ng a power of two in [8, 1024], n > 0, box > 0, known flags, "
                "non-NULL pointers");
  if ((size_t)ws_bytes < pk_workspace_bytes(ng))
    return fail(nullptr, SDPM_ENOMEM, "power_spectrum: workspace of %lld bytes < %zu required",
                (long long)ws_bytes, pk_workspace_bytes(ng));
  char msg[256] = {0};
  const int rc = power_spectrum(x_dev, n, box, ng, flags, workspace, (hipStream_t)hip_stream, k, p,
                                p_raw, modes, msg, sizeof msg);
  return rc ? fail(nullptr, rc, "power_spectrum: %s", msg) : SDPM_OK;
}

int sdpm_net_scratch_bytes(int32_t n, int64_t* bytes) {
  if (!net_size_ok(n) || !bytes) return fail(nullptr, SDPM_EINVAL, "n must be a power of two >= 16");
  *bytes = (int64_t)net_train_scratch_bytes(n);
  return SDPM_OK;
}

int sdpm_conv3d_wgrad(int32_t n, const void* in_bf16, const void* g_bf16, float* dw, float* db,
                      void* scratch, int64_t scratch_bytes, void* stream) {
  if (!net_size_ok(n) || !in_bf16 || !g_bf16 || !dw || !db || !scratch)
    return fail(nullptr, SDPM_EINVAL, "conv3d_wgrad: bad arguments");
  if ((size_t)scratch_bytes < wgrad_scratch_bytes(n))
    return fail(nullptr, SDPM_ENOMEM, "conv3d_wgrad: scratch too small");
  launch_conv_wgrad(n, (const uint16_t*)in_bf16, (const uint16_t*)g_bf16, dw, db, (float*)scratch,
                    (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "wgrad launch failed");
}

int sdpm_net_prep(int32_t n, const float* r, const float* phi, float s_r, float s_phi,
                  float kappa_h2, void* act0, void* stream) {
  if (!net_size_ok(n) || !r || !phi || !act0) return fail(nullptr, SDPM_EINVAL, "net_prep: bad arguments");
  launch_net_prep<float, float, false>(n, r, phi, s_r, s_phi, kappa_h2, nullptr, (uint16_t*)act0,
                                       (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "net_prep launch failed");
}

int sdpm_net_forward(int32_t n, const float* params, const void* act0, void* act_a, void* act_b,
                     float* out, void* stream) {
  if (!net_size_ok(n) || !params || !act0 || !act_a || !act_b || !out)
    return fail(nullptr, SDPM_EINVAL, "net_forward: bad arguments");
  net_forward(n, params, (const uint16_t*)act0, (uint16_t*)act_a, (uint16_t*)act_b, out,
              (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "net_forward failed");
}

// Allocation-free net forward.  The two hidden-layer activation buffers live
// in `scratch`, a file-scope device array of two kNoAllocMaxN^3 x 16 BF16
// buffers (16 MiB), of which each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, on the entry point's first call there, and kept.
namespace {
constexpr int kNoAllocMaxN = 64;
constexpr size_t kNoAllocActBytes =
    (size_t)kNoAllocMaxN * kNoAllocMaxN * kNoAllocMaxN * 16 * sizeof(uint16_t);
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[2 * kNoAllocActBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return fail(nullptr, SDPM_EHIP, "net_forward_noalloc: hipGetSymbolAddress failed");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SDPM_OK;
}
}  // namespace

int sdpm_net_forward_noalloc(int32_t n, const float* params, const void* act0, float* out,
                             void* stream) {
  if (!net_size_ok(n) || !params || !act0 || !out)
    return fail(nullptr, SDPM_EINVAL, "net_forward_noalloc: bad arguments");
  if (n > kNoAllocMaxN)
    return fail(nullptr, SDPM_EINVAL,
                "net_forward_noalloc: n = %d exceeds the static scratch (n <= %d)", n,
                kNoAllocMaxN);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(nullptr, SDPM_EHIP, "net_forward_noalloc: no current device below %d",
                kNoAllocMaxDevices);
  void* base = nullptr;
  const int rc = scratch_address(dev, &base);
  if (rc) return rc;
  uint16_t* act_a = (uint16_t*)base;
  uint16_t* act_b = (uint16_t*)((char*)base + kNoAllocActBytes);
  net_forward(n, params, (const uint16_t*)act0, act_a, act_b, out, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK
                                         : fail(nullptr, SDPM_EHIP, "net_forward_noalloc failed");
}

int sdpm_net_train_step(int32_t n, float* params, float* m1, float* m2, int32_t step, float lr,
                        const void* act0, const float* target, float target_scale, void* scratch,
                        int64_t scratch_bytes, float* loss_dev, void* stream) {
  if (!net_size_ok(n) || !params || !m1 || !m2 || !act0 || !target || !scratch || !loss_dev ||
      step < 1 || !(lr > 0.f))
    return fail(nullptr, SDPM_EINVAL, "net_train_step: bad arguments");
  if ((size_t)scratch_bytes < net_train_scratch_bytes(n))
    return fail(nullptr, SDPM_ENOMEM, "net_train_step: scratch too small");
  net_train_step(n, params, m1, m2, step, lr, (const uint16_t*)act0, target, target_scale, scratch,
                 loss_dev, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SDPM_OK : fail(nullptr, SDPM_EHIP, "train step failed");
}

int sdpm_profile(sdpm_ctx* c, int32_t enable) {
  if (!c) return SDPM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  c->prof.reset();
  c->prof.on = enable != 0;
  c->prof.mask = ~0ull;
  return SDPM_OK;
}

int sdpm_profile_kernels(sdpm_ctx* c, const char* names) {
  if (!c) return SDPM_EINVAL;
  if (!names) return fail(c, SDPM_EINVAL, "names must not be NULL");
  uint64_t mask = 0;
  const char* p = names;
  while (*p) {
    const char* q = std::strchr(p, ',');
    const size_t len = q ? (size_t)(q - p) : std::strlen(p);
    int id = -1;
    for (int k = 0; k < K_NKERNELS; ++k)
      if (std::strlen(kKernelNames[k]) == len && std::strncmp(kKernelNames[k], p, len) == 0) id = k;
    if (id < 0) return fail(c, SDPM_EINVAL, "unknown kernel name '%.*s'", (int)len, p);
    mask |= 1ull << id;
    if (!q) break;
    p = q + 1;
  }
  if (!mask) return fail(c, SDPM_EINVAL, "no kernel named");
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  c->prof.reset();
  c->prof.on = true;
  c->prof.mask = mask;
  return SDPM_OK;
}

int sdpm_profile_read(sdpm_ctx* c, sdpm_kernel_stat* out, int32_t max, int32_t* n) {
  if (!c || !n || (max > 0 && !out)) return SDPM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->st));
  if (c->prof.on) c->prof.collect();
  *n = K_NKERNELS;
  for (int k = 0; k < K_NKERNELS && k < max; ++k) {
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, kKernelNames[k], sizeof(out[k].name) - 1);
    out[k].launches = c->prof.launches[k];
    out[k].ms = c->prof.ms[k];
    out[k].bytes = c->prof.bytes[k];
  }
  return SDPM_OK;
}

int sdpm_destroy(sdpm_ctx* c) {
  if (!c) return SDPM_OK;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  c->prof.release();
  fft_destroy(&c->fft);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipHostFree(c->hpin);
  delete c;
  return SDPM_OK;
}

const char* sdpm_last_error(const sdpm_ctx* c) { return c ? c->err : g_create_err; }

}  // extern "C"
