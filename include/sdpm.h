/*
 * sdpm.h - C ABI of the shrinking-domain particle-mesh library (libsdpm.so).
 *
 * One step of the particle-mesh method of Llinares (2017), "The shrinking
 * domain framework I", on one AMD Instinct MI355X (gfx950):
 *   Sec. 2.2 Eqs. 7-9  synchronised leapfrog (drift 1/2, kick, drift 1/2);
 *   Sec. 2.4           CIC mass deposit and CIC force interpolation with the
 *                      same weights (momentum conservation);
 *   Sec. 2.1 Eqs. 3-4  gravity: Poisson (static) or the diffusion equation,
 *                      advanced here by one implicit (backward Euler) step per
 *                      half sub-step, both solved by multigrid;
 *   Sec. 2.3 Table 2   ordering of operations within a step;
 *   Sec. 2.4 Eq. 10    lightcone of the z = 0 observer; particles outside it
 *                      are eliminated and the active cells shrink to an index
 *                      box; Sec. 3: periodic until that box fits in the mesh.
 *
 * Units: comoving Mpc/h, conformal time in 1/H0 (H0 = 1), so the speed of
 * light is 2997.92458.  Momentum p = a dx/dtau.  The mesh equation in grid
 * units is (Lap_h - kappa h^2) Phi = h^2 (S delta - kappa Phi_old), with the
 * 7-point Laplacian, S = 3 Omega_m / (2 a), kappa = 3 calH / (c_g^2 dtau/2).
 *
 * Conventions for every call:
 *  - Return value: SDPM_OK (0) or a negative SDPM_E* code.  No call throws or
 *    aborts across the ABI.  sdpm_last_error() describes the last failure on
 *    a context.  An error other than SDPM_EHIP leaves the context usable and
 *    its state consistent (what a failing call has completed is stated with
 *    the call).  SDPM_EHIP reports a failed HIP runtime call: the device
 *    state is then undefined (a step may have been applied in part) and the
 *    context should be destroyed.
 *  - Device buffers (particles, fields, workspace) are caller-owned device
 *    memory that the context borrows; they must outlive the context.
 *  - All device work is enqueued on the stream given to sdpm_create.  Calls
 *    that return host scalars synchronise that stream before returning.
 *  - One context per stream; a context is not thread-safe.
 *  - Mesh layout: cell (i, j, k) at linear index (k ng + j) ng + i, value at
 *    position (i h, j h, k h), h = box / ng.  Particle arrays are SoA.
 */
#ifndef SDPM_H
#define SDPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SDPM_OK = 0,
  SDPM_EINVAL = -1,     /* invalid argument or configuration            */
  SDPM_ENOMEM = -2,     /* workspace too small / host allocation failed */
  SDPM_EHIP = -3,       /* a HIP runtime call failed                     */
  SDPM_ENOCONV = -4,    /* multigrid did not reach tol in max_outer      */
  SDPM_EDOMAIN = -5,    /* a particle's CIC support left the active box  */
  SDPM_EOVERFLOW = -6,  /* fixed-point coordinate out of range           */
  SDPM_ESTATE = -7,     /* call out of order (e.g. step before bind)     */
  SDPM_EFULL = -8       /* lightcone output full: later records dropped  */
};

enum { SDPM_MIXED = 0, SDPM_PLAIN_FP64 = 1 };      /* sdpm_config.precision  */
/* sdpm_config.warm_start.  PREV: the previous potential.  LEARNED: the
 * learned guess (below) before every solve.  LEARNED_GATED: the learned
 * guess only while it pays: per sub-step kind (first / second field
 * half-step) the context times the guess and one V-cycle (with its share of
 * the defect-correction passes) with HIP events and estimates the V-cycles an
 * accepted guess saved (its residual reduction in units of the solve's
 * measured convergence factor per cycle);
 * when the saving is below the cost, the next B * max(1, cost / saving)
 * solves of that kind skip the net, B = 8, 16, 32, ... (doubling at each
 * failed try), at most 256.                                                */
enum { SDPM_WS_PREV = 0, SDPM_WS_LEARNED = 1, SDPM_WS_LEARNED_GATED = 2 };
/* Flag OR-ed into warm_start: start each solve of sdpm_step from the
 * potential plus the change that the same solve (first or second field
 * half-step) made in the previous step, scaled by the ratio of the conformal
 * steps (linear extrapolation in time; the first step of a run starts from
 * the previous potential).  Costs two passes over the active box per solve
 * (an FP32 copy of the start, then the change) and three FP32 meshes.
 * Applied while the mesh is periodic; on the frozen-exterior box solves
 * start from the previous potential (the extrapolation saved no iteration
 * there).                                                                  */
enum { SDPM_WS_EXTRAP = 4 };
/* sdpm_config.solver: how each half sub-step advances the potential by the
 * diffusion equation of Sec. 2.1 Eq. 4.  SDPM_SOLVER_IMPLICIT: one backward-
 * Euler step solved by multigrid to tol.  SDPM_SOLVER_ADE: the paper's own
 * alternating-direction explicit integrator (Sec. 2.3): one Saul'yev sweep
 * per half sub-step, forward for the first and backward for the second (see
 * sdpm_ade_sweep); needs a finite gravity speed (c_grav != 0) and
 * warm_start == SDPM_WS_PREV, and leaves the step's outer_iters and
 * residuals at 0.  The initial static solve is multigrid in both cases.    */
/* SDPM_SOLVER_FFT: the implicit step (and the initial static solve) solved
 * exactly by FFT while the mesh is periodic (the standard particle-mesh
 * solver the paper compares against, Sec. 2.4, with the 7-point symbol),
 * multigrid once the domain has a frozen exterior; FP64 hipFFT transforms
 * with their work area in the workspace; needs warm_start == SDPM_WS_PREV;
 * reports 0 iterations and residual 0 for FFT solves.                      */
enum { SDPM_SOLVER_IMPLICIT = 0, SDPM_SOLVER_ADE = 1, SDPM_SOLVER_FFT = 2 };
/* sdpm_config.assignment.  CIC: the 2^3 cells around a particle, axis
 * weights (2^B - q, q) of the fixed-point coordinate U = floor(x s),
 * q = U mod 2^B.  TSC: the 3^3 nodes around the nearest node
 * i = (U + 2^(B-1)) >> B; with D = U - i 2^B the outer axis weights are
 * (2^(B-1) -+ D)^2 / 2^(B+1) rounded to the nearest integer and the middle
 * one 2^B minus both.  Either way the products sum to 2^(3B) exactly, the
 * deposit is exact integer arithmetic, and the active box must hold the
 * whole support (one node more on each side for TSC).                      */
enum { SDPM_ASSIGN_CIC = 0, SDPM_ASSIGN_TSC = 1 };

typedef struct sdpm_ctx sdpm_ctx;                  /* opaque */

typedef struct sdpm_config {
  int32_t ng;            /* mesh cells per axis: power of two, 8..2048          */
  int32_t frac_bits;     /* B, fractional bits of the CIC coordinate (1..16)    */
  double box;            /* comoving box side L [Mpc/h]                         */
  double omega_m, omega_l;
  double c_light;        /* speed of light, 2997.92458 in these units          */
  double c_grav;         /* 0: static Poisson; < 0: 0.019 h c (Sec. 3.1.1,
                            Eq. 12, h in Mpc/h); > 0: this speed              */
  double x_obs[3];       /* observer position [Mpc/h]                          */
  int32_t shrink;        /* 0: fixed periodic domain; 1: shrinking domain      */
  int32_t margin;        /* cells added around the lightcone sphere (>= 2;
                            TSC assignment adds one more, see
                            sdpm_domain_box)                                   */
  int32_t box_align;     /* power of two A: the planes next to the active box
                            sit at multiples of A (A = 2^(mg_levels-1) nests
                            every multigrid level exactly)                     */
  int32_t mg_levels;     /* multigrid levels incl. the finest (>= 2), at most:
                            a V-cycle ends on the first coarser level whose
                            own red-black sweeps cut its slowest mode by 1e-3
                            in at most pre + post + 1 sweeps (kappa h^2 > 0
                            makes the coarse diagonals dominant)             */
  int32_t pre, post;     /* RB Gauss-Seidel sweeps before / after coarse work  */
  int32_t coarse_sweeps; /* max RB Gauss-Seidel sweeps on the coarsest level   */
  int32_t max_outer;     /* FP64 defect-correction iterations per solve        */
  double tol;            /* stop when ||r||_2 <= tol ||rhs||_2 (active cells)  */
  int32_t precision;     /* SDPM_MIXED: FP32 V-cycles in FP64 defect
                            correction, FP32 momenta; SDPM_PLAIN_FP64: FP64
                            V-cycles and momenta                               */
  int32_t warm_start;    /* SDPM_WS_PREV, SDPM_WS_LEARNED(_GATED), | EXTRAP    */
  int64_t n_initial;     /* particles at the start: mean density n0 / ng^3     */
  int32_t sort_every;    /* Morton re-sort before every k-th step (0: never)   */
  int32_t sort_shift;    /* sort key: Morton order of cell blocks of 2^shift
                            cells per axis, then the cell row (z, then y)
                            inside the block (stable: particles keep their
                            order inside a row); default 4 for ng >= 64      */
  int32_t solver;        /* SDPM_SOLVER_IMPLICIT (default), _ADE or _FFT        */
  int32_t cycles_per_outer; /* V-cycles per defect-correction iteration, at most
                            (1..4, default 4): further cycles on the same
                            defect equation while fewer are predicted (from
                            the last solve's factor per cycle) to leave the
                            residual above tol and their combined factor
                            stays well above the rounding floor of the
                            stored correction; the result meets tol either
                            way                                              */
  int32_t assignment;    /* SDPM_ASSIGN_CIC (default) or SDPM_ASSIGN_TSC: the
                            mass assignment and force interpolation scheme
                            (Sec. 2.4 names both; the same weights both ways) */
} sdpm_config;

/* Caller-owned device arrays.  x: FP64 positions in [0, box); p: momenta,
 * float when precision == SDPM_MIXED, double when SDPM_PLAIN_FP64; id: any
 * labels.  Entries [0, n_active) are the active particles; removed particles
 * are kept after them in removal order (stable partition).                  */
typedef struct sdpm_particles {
  double* x[3];
  void* p[3];
  uint32_t* id;
  int64_t capacity;
} sdpm_particles;

/* Caller-owned device mesh arrays, ng^3 each.  phi: potential (in/out): a
 * step reads it as Phi_old (the previous potential of Eq. 4's implicit
 * step and the solve's initial guess) and overwrites it in place with
 * Phi(t + dt/2), then Phi(t + dt); rhs: right-hand side of the last solve
 * (out); counts: fixed-point CIC mass of the last deposit, sum over a
 * particle's cells = 2^(3B) (out).  The force -grad Phi has no caller
 * array: in mixed precision the step writes it to an FP32 mesh in the
 * workspace (3 values per cell), in plain FP64 the interpolation
 * differences phi at each node.                                             */
typedef struct sdpm_fields {
  double* phi;
  double* rhs;
  uint64_t* counts;
} sdpm_fields;

typedef struct sdpm_step_stats {
  int64_t n_active, n_removed;
  int32_t outer_iters[2];  /* per field sub-step (second is 0 if static)  */
  int32_t vcycles;         /* V-cycles in this call                       */
  int32_t warm_used;       /* 1 if the learned guess was accepted         */
  double res0[2], res[2];  /* relative residual before / after each solve
                              (after: the FP64 residual, or where the last
                              correction's estimate r_old - A e with its
                              rounding bound settled convergence, that
                              estimate, within the bound of it) */
  double dtau, a_half, kappa_h2[2], r_lc;
  int32_t lo[3], hi[3], periodic;
  float ms[8];             /* [0] drift+deposit [1] rhs [2] solve 1
                              [3] force+kick+drift [4] solve 2
                              [5] removal+compaction [6] total           */
  double res_guess[2];     /* relative residual of the accepted initial
                              guess (equal to res0 when the learned guess
                              was not used)                              */
} sdpm_step_stats;

/* Host-only scalars of one step a -> a + da (no device work):
 * out[0] dtau, [1] a_half (conformal midpoint), [2] S(a_half),
 * [3] kappa_1 h^2, [4] kappa_2 h^2, [5] lightcone radius at a + da,
 * [6] gravity speed c_g.  Sec. 2.2 Eqs. 7-9, Sec. 2.4 Eq. 10 (read as the
 * light travel distance from a to today, shrinking to 0 at a = 1).        */
int sdpm_step_scalars(const sdpm_config* cfg, double a, double da, double out[7]);

/* Lightcone radius at a (host only).                                        */
int sdpm_lightcone_radius(const sdpm_config* cfg, double a, double* r);

/* Active index box for lightcone radius r (host only), Sec. 2.4: cells
 * within r + m cells of the observer per axis, m = margin (CIC) or
 * margin + 1 (TSC, whose support reaches one node further),
 *   lo0 = floor((x_o - r)/h) - m,  hi0 = floor((x_o + r)/h) + m,
 * rounded outward so that lo - 1 and hi + 1 are multiples of box_align.  periodic
 * = 1 (and the box is the whole mesh) while that box does not fit in
 * [1, ng - 2]; lo/hi are inclusive, axis order x, y, z.                     */
int sdpm_domain_box(const sdpm_config* cfg, double r, int32_t lo[3], int32_t hi[3],
                    int32_t* periodic);

/* Fills cfg with defaults for mesh ng and box L (MG min(6, log2(ng) - 1)
 * levels, V(2,2), 64 coarse sweeps, tol 1e-8, B = 14, margin 2, box_align
 * 2^(levels-1), observer at the centre, static gravity, no shrinking).     */
int sdpm_config_default(sdpm_config* cfg, int32_t ng, double box);

/* Device workspace needed for `capacity` particles.                         */
int sdpm_workspace_bytes(const sdpm_config* cfg, int64_t capacity, int64_t* bytes);

/* Creates a context.  workspace: caller-owned device memory of at least
 * sdpm_workspace_bytes; hip_stream: hipStream_t (NULL = default stream).
 * The library allocates only a small host buffer for scalars.              */
int sdpm_create(const sdpm_config* cfg, void* workspace, int64_t ws_bytes,
                void* hip_stream, sdpm_ctx** out);

/* "Init particles": borrows the particle and field arrays; n_active
 * particles are live.  Resets the domain to periodic / whole mesh.          */
int sdpm_bind(sdpm_ctx* ctx, const sdpm_particles* parts, const sdpm_fields* fields,
              int64_t n_active);

/* "Init domain": applies the lightcone at a (removing particles outside it
 * when shrinking), then sets phi by one static (kappa = 0) solve of the
 * density at a (Table 1: field initial conditions from linear theory).      */
int sdpm_init_potential(sdpm_ctx* ctx, double a, sdpm_step_stats* out);

/* One step a -> a + da in the order of Table 2: drift dtau/2 with a (Eq. 7),
 * CIC deposit, solve to a_half, FD force, CIC interpolation, kick with
 * a_half (Eq. 8), drift dtau/2 with a + da (Eq. 9), second field half
 * sub-step (skipped for static gravity), lightcone and elimination at
 * a + da.  The deposit reads the drifted positions without storing them;
 * the interpolation pass evaluates the same first drift again and stores
 * only the positions at a + da.  out may be NULL.  Errors: SDPM_EINVAL /
 * SDPM_ESTATE before any device work (nothing changed); SDPM_ENOCONV,
 * SDPM_EDOMAIN, SDPM_EOVERFLOW and SDPM_EFULL after the whole step has been
 * applied (positions, momenta, potential and time advanced; ENOCONV keeps
 * the best iterate of the solve that missed tol; with EDOMAIN / EOVERFLOW
 * the offending particles took the first drift only, without deposit, kick
 * or second drift, and the lightcone is not applied in that step: no
 * particle removed, the domain not shrunk); SDPM_EHIP as above (a failure
 * in the first solve returns before the kick, with positions and momenta
 * as they were at a).                                                      */
int sdpm_step(sdpm_ctx* ctx, double a, double da, sdpm_step_stats* out);

/* "Shrink domain": lightcone at a; stable-partitions the active particles
 * (outside ones after the kept ones), writes their ids to removed_ids_dev
 * (device, may be NULL) and updates the active box.  Sec. 2.4, Table 2.     */
int sdpm_shrink(sdpm_ctx* ctx, double a, int64_t* n_removed, uint32_t* removed_ids_dev);

/* As sdpm_shrink but with an explicit lightcone radius r (for tests).       */
int sdpm_shrink_radius(sdpm_ctx* ctx, double r, int64_t* n_removed,
                       uint32_t* removed_ids_dev);

/* Lightcone output ----------------------------------------------------------
 * The natural output of the method is the past lightcone of the observer
 * (Sec. 1 list of the framework's characteristics; Table 2 last row: the
 * particles leaving the lightcone are eliminated).  When enabled, every
 * particle removed by sdpm_step is recorded where it crosses the lightcone
 * during that step: traced back from its end-of-step position x1 along its
 * end-of-step velocity, x(u) = x1 - u w with w = p1 dtau / a1, while the
 * lightcone radius grows back as r(u) = r1 + u c dtau (r_lc is linear in
 * conformal time), u in [0, 1] the fraction of the step before its end; the
 * crossing is the root of |x(u) - x_obs| = r(u) (u = 1, the step's start,
 * for a particle that was already outside then).  Record: id, a = a1 - u da,
 * x(u), p1.  sdpm_shrink(a) and sdpm_init_potential record their removals
 * at u = 0; sdpm_shrink_radius records nothing.  Records are appended in
 * removal order (the order of the stable partition); once `capacity` is
 * reached later records are dropped and the call returns SDPM_EFULL after
 * completing its work.  Device arrays of `capacity` entries, caller-owned.
 * On a fixed domain (shrink == 0) nothing is removed: sdpm_step records the
 * particles that cross the lightcone during the step, those outside at its
 * end (the removal test with r_lc(a + da)) that were inside at its start
 * (the same test with the previous step's end radius, or r_lc(a) for the
 * first step), with the same crossing formula; they stay in the simulation
 * and the records of one step come in no particular order.  This is the
 * lightcone of the run without shrinking that the paper compares against. */
typedef struct sdpm_lightcone {
  uint32_t* id;
  double* a;
  double* x[3];
  double* p[3];
  int64_t capacity;
} sdpm_lightcone;
/* Enables the output into `out` (NULL disables) and resets the count.      */
int sdpm_set_lightcone(sdpm_ctx* ctx, const sdpm_lightcone* out);
/* Records written since sdpm_set_lightcone.                                */
int sdpm_lightcone_count(sdpm_ctx* ctx, int64_t* count);

/* Current state: n_active, box, boundary mode (host scalars).              */
int sdpm_get_state(sdpm_ctx* ctx, sdpm_step_stats* out);

/* Sub-steps for kernel-level checks --------------------------------------- */
/* Mass assignment of Sec. 2.4 (CIC, or TSC when sdpm_config.assignment
 * selects it; the same weights as the interpolation): the active particles
 * at their current positions (no drift) into fields->counts, which is
 * zeroed first over the active box (the whole mesh while periodic).  Fixed
 * point: U = floor(x ng 2^B / box) per axis, CIC axis weights (2^B - q, q)
 * of the cells U >> B and (U >> B) + 1, q = U mod 2^B; the weight products
 * (<= 2^(3B)) are summed exactly in uint64, so every particle adds 2^(3B).
 * Errors: SDPM_ESTATE before sdpm_bind; SDPM_EDOMAIN when a particle's
 * support leaves the active box, SDPM_EOVERFLOW for a non-finite
 * coordinate (those particles are skipped, the others deposited).          */
int sdpm_deposit(sdpm_ctx* ctx);
/* Source and mesh solve of one implicit half sub-step of Eq. 4 (Sec. 2.1;
 * kappa = 0 is Poisson's equation, Eq. 3), from the last deposit:
 *   rhs = h^2 S (counts / (n0/ng^3 2^3B) - 1) [- its mean while periodic]
 *         - kappa h^2 phi,
 * then (Lap_h - kappa h^2) phi = rhs on the active box (7-point Laplacian
 * in grid units, frozen exterior values once the box is smaller than the
 * mesh, zero mean for periodic kappa = 0) by the configured solver, phi
 * (fields->phi, in/out) as the initial guess, to the relative residual
 * sdpm_config.tol.  kappa_h2 = kappa h^2 >= 0; s_h2_factor = S (the factor
 * 3 Omega_m / (2 a) of Eq. 3; h^2 is applied inside).  fields->rhs receives
 * the right-hand side.  Errors: SDPM_EINVAL for kappa_h2 < 0 or a non-finite
 * argument; SDPM_ENOCONV when max_outer corrections do not reach tol (phi
 * holds the last iterate, out->res its residual).                           */
int sdpm_solve(sdpm_ctx* ctx, double kappa_h2, double s_h2_factor, sdpm_step_stats* out);
/* One ADE sweep (Sec. 2.3) of fields->phi in place over the active box with
 * fields->rhs as the source f = S h^2 delta (the caller's values; sdpm_step
 * assembles it):  (1 + 3 lam) phi_c' = (1 - 3 lam) phi_c + lam (S6 - f_c),
 * S6 the six neighbours' current values, cells visited in lexicographic order
 * (forward != 0: z, y, x increasing; 0: decreasing), so neighbours visited
 * earlier enter with their new values.  Periodic wrap while the mesh is
 * periodic; frozen exterior otherwise.  lam = D dt / h^2 > 0 (sdpm_step uses
 * 1 / kappa_h2 of the half sub-step).  Runs on the context's stream, one
 * launch per diagonal of rows (ny + nz - 1 launches).  SDPM_EINVAL for lam
 * not finite and positive.                                                  */
int sdpm_ade_sweep(sdpm_ctx* ctx, double lam, int forward);
/* The multigrid smoother of the implicit solve (Sec. 2.1 Eq. 4) on one
 * periodic FP32 level: four red-black Gauss-Seidel half sweeps (red, black,
 * red, black) of (Lap - kappa) e = scale r in colour-split storage (the
 * n^3/2 red cells, (i+j+k) even, first, then the black ones, each in
 * (k, j, i >> 1) row order), each cell set to
 *   e = (sum of its 6 neighbours - scale r) * inv_diag
 * with inv_diag = 1 / (6 + kappa h^2 scale).  first != 0: the red sweep
 * starts from e = 0 (e is not read and may be NULL).  fused != 0: one
 * z-marching pass that keeps the sweeps' planes in LDS (what the V-cycle
 * runs on levels of at least 256^3 cells), reading e and writing e_out,
 * which must differ unless first; fused == 0: e copied to e_out (unless
 * first or the same) and four single-colour launches in place on e_out.
 * Both forms give bit-identical e_out.  n: power of two in [64, 2048]; all
 * arrays device memory of n^3 floats; runs on stream (hipStream_t, NULL =
 * default), asynchronously.  SDPM_EINVAL for other sizes, NULL pointers or
 * e == e_out with fused and not first.  t_out (NULL for none): the red
 * residual of the result, t = r - (sum of the 6 neighbours - 6 e) / scale +
 * kappa_h2 e (kappa_h2 = kappa h^2 of the finest level: inv_diag =
 * 1 / (6 + kappa_h2 scale)), the V-cycle's restriction input, into the red
 * half of t_out (n^3 floats; the black half is not written); the fused form
 * then does not write the red half of e_out (the V-cycle does not read it
 * before the post-smoothing sets it anew), the other writes it and t_out by
 * a separate launch; t_out's red half and e_out's black half are
 * bit-identical between the two.  box (NULL: the periodic whole mesh):
 * lo[3], hi[3] of a frozen-exterior box (the shrinking domain's index box,
 * Sec. 2.4), 1 <= lo <= hi <= n - 2 per axis; e is zero outside it and stays
 * zero (the correction's homogeneous Dirichlet condition), only its cells
 * are swept.  SDPM_EINVAL also for t_out with scale <= 0 or aliasing another
 * array, or a box that reaches a face of the mesh.                         */
int sdpm_rb_sweeps(int32_t n, const float* e, float* e_out, const float* r, float scale,
                   float inv_diag, int32_t first, int32_t fused, float* t_out, float kappa_h2,
                   const int32_t* box, void* stream);
/* Re-sort of the active particles (all SoA arrays permuted together by the
 * key of sort_shift: the Morton code of the cell's block, then its row
 * inside the block; stable LSD radix sort).  Results of the step do not
 * depend on particle order (only the order of removed particles and of
 * lightcone records follows it); the sort improves locality.              */
int sdpm_sort(sdpm_ctx* ctx);
/* Force interpolation of Sec. 2.4 with the deposit's own weights (the same
 * scheme both ways, which conserves momentum): g = -grad Phi by central
 * differences of fields->phi, (Phi_{i+1} - Phi_{i-1}) / (2h) per axis, at
 * each assignment node, weighted and summed per active particle (FP64).
 * g_dev[3]: caller-owned device FP64 arrays of n_active entries (x, y, z
 * components), written in the particles' current order.  Errors: as
 * sdpm_deposit (an offending particle's entries are left unwritten).       */
int sdpm_interp_force(sdpm_ctx* ctx, double* g_dev[3]);

/* Power spectrum ------------------------------------------------------------
 * The accuracy metric the paper compares runs with (Sec. 3.1, Sec. 3.2: 3D
 * spectra of the lightcone in a cubical box of the original size), with the
 * discreteness corrections of Jing (2005) that the paper names for its
 * spectrum tool (Sec. 2.4).  Standalone: no context.
 * x_dev[3]: device FP64 positions of n particles, each in [0, box] (box is
 * the periodic image of 0, as in the step's deposit); ng: mesh
 * of the estimate, a power of two in [8, 1024].  delta from the fixed-point
 * CIC counts (B = 14), one FP64 FFT, shells b = rint(|f|) = 1 .. ng/2 of the
 * signed integer frequency f (k = f 2 pi / box).  Per shell (host arrays of
 * ng/2): k = mean |k| of its modes [h/Mpc], modes, p_raw = mean of
 * box^3 |delta_k|^2 (delta_k = FFT / ng^3), and p:
 *   p_raw - shot <C1>              without SDPM_PK_JING,
 *   (p_raw - shot <C1>) / <S>      with it (Jing's alias correction),
 * shot = box^3 / n with SDPM_PK_SHOT, else 0; C1(f) = prod_d (1 - 2/3
 * sin^2(pi f_d / ng)); S(f) = sum over images m in [-2, 2]^3 of
 * prod_d sinc^4(pi (f_d + ng m_d) / ng) (|f + ng m| / |f|)^neff, neff the
 * shell's local log-log slope of p, starting at 0 and re-estimated three
 * times (central differences of neighbouring shells, one-sided at the ends,
 * clamped to [-4, 4], 0 where a neighbour is not positive).
 * workspace: device memory of sdpm_pk_workspace_bytes(ng); runs on
 * hip_stream and returns when the results are on the host (the FFT plan is
 * made per call).  Errors: SDPM_EINVAL (arguments), SDPM_ENOMEM (workspace
 * too small), SDPM_EDOMAIN (a position outside [0, box]), SDPM_EHIP.     */
enum { SDPM_PK_SHOT = 1, SDPM_PK_JING = 2 };
int sdpm_pk_workspace_bytes(int32_t ng, int64_t* bytes);
int sdpm_power_spectrum(const double* const x_dev[3], int64_t n, double box, int32_t ng,
                        int32_t flags, void* workspace, int64_t ws_bytes, void* hip_stream,
                        double* k, double* p, double* p_raw, int64_t* modes);

/* Learned warm start ------------------------------------------------------
 * Not in the paper: a learned initial guess for the multigrid solve of each
 * implicit gravity sub-step.  A 5-layer 3x3x3 convolution net, 16 channels,
 * ReLU between layers, periodic padding on the ng^3 mesh, BF16 weights and
 * activations with FP32 accumulation on the matrix cores.  Input channels:
 * the residual of the previous potential r0 = rhs - A phi_old (the density
 * source minus the Laplacian of phi_old) scaled by 1/rms(r0), and phi_old
 * scaled by 1/rms(phi_old), and the constant kappa h^2 of the sub-step (the
 * change solves (A) dphi = r0, whose kernel depends on kappa h^2 only).
 * Output: the change of the potential in units of
 * 1/rms(r0).  The guess replaces phi_old only if its residual is smaller;
 * the solve always continues to tol, so plain multigrid decides the result and
 * the fallback.
 * Parameters: SDPM_NET_PARAMS FP32 values, per layer l = 0..4 the weights
 * W[t][ci][co] (27 x 16 x 16, tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) reading
 * the input at (i+dx, j+dy, k+dz)) then the bias b[co] (16); input channels
 * ci >= 3 of layer 0 and output channels co >= 1 of layer 4 are unused.
 * Activations: ng^3 x 16 BF16 (uint16), channels fastest, voxel (i,j,k) at
 * (k ng + j) ng + i.  Device pointers; work is enqueued on `stream`.        */
#define SDPM_NET_PARAMS (5 * (27 * 16 * 16 + 16))
enum { SDPM_CONV_RELU = 1, SDPM_CONV_OUT_FP32_CH0 = 2, SDPM_CONV_BACKWARD_DATA = 4,
       SDPM_CONV_MASK = 8 };
/* Loads FP32 parameters (host memory, n_params == SDPM_NET_PARAMS) into a
 * context created with warm_start = SDPM_WS_LEARNED or _LEARNED_GATED.    */
int sdpm_set_warmstart_weights(sdpm_ctx* ctx, const float* params_host, int64_t n_params);
/* One convolution layer (flags: SDPM_CONV_*):
 *   out[v][co] = bias[co] + sum_t sum_ci in[v + off_t][ci] W[t][ci][co],
 * then ReLU; with BACKWARD_DATA the adjoint (mirrored taps, W transposed,
 * no bias): out[u][ci] = sum_t sum_co in[u - off_t][co] W[t][ci][co], then
 * times [mask > 0] with MASK (mask: BF16 activations).  out: BF16 ng^3 x 16,
 * or FP32 ng^3 (channel 0) with OUT_FP32_CH0.  n: power of two >= 16.      */
int sdpm_conv3d(int32_t n, const void* in_bf16, const float* w, const float* bias, int32_t flags,
                const void* mask_bf16, void* out, void* stream);
/* Weight and bias gradients of sum(out * g) for out = conv(in):
 * dw[t][ci][co] = sum_v in[v + off_t][ci] g[v][co], db[co] = sum_v g[v][co];
 * summed in a fixed order (deterministic).  scratch: sdpm_net_scratch_bytes. */
int sdpm_conv3d_wgrad(int32_t n, const void* in_bf16, const void* g_bf16, float* dw, float* db,
                      void* scratch, int64_t scratch_bytes, void* stream);
/* Device scratch needed by sdpm_conv3d_wgrad and sdpm_net_train_step.      */
int sdpm_net_scratch_bytes(int32_t n, int64_t* bytes);
/* act0[v] = (r[v] s_r, phi[v] s_phi, kappa_h2, 0, ..., 0) in BF16; r, phi
 * FP32 ng^3.                                                               */
int sdpm_net_prep(int32_t n, const float* r, const float* phi, float s_r, float s_phi,
                  float kappa_h2, void* act0, void* stream);
/* Net forward: out (FP32 ng^3) = channel 0 of layer 5; act_a / act_b: two
 * BF16 ng^3 x 16 buffers for the hidden layers.                            */
int sdpm_net_forward(int32_t n, const float* params, const void* act0, void* act_a, void* act_b,
                     float* out, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the net
 * forward of sdpm_net_forward, same kernels and the same result, with the
 * two hidden-layer buffers taken from a static device array inside the
 * library (16 MiB per GPU, held until the process ends) instead of act_a /
 * act_b.  It calls no allocating routine.  n: a power of two in [16, 64]
 * (SDPM_EINVAL beyond 64: the array's size); params, act0, out and stream as
 * for sdpm_net_forward.  Every call on one GPU uses that GPU's one array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller.                                    */
int sdpm_net_forward_noalloc(int32_t n, const float* params, const void* act0, float* out,
                             void* stream);
/* One training step on one sample: forward, loss = mean((out - target_scale
 * target)^2)
 * written to *loss_dev (device FP32), backward through all layers, Adam
 * (beta 0.9 / 0.999, step counted from 1) on params with moments m1, m2.   */
int sdpm_net_train_step(int32_t n, float* params, float* m1, float* m2, int32_t step, float lr,
                        const void* act0, const float* target, float target_scale, void* scratch,
                        int64_t scratch_bytes, float* loss_dev, void* stream);
/* Records every multigrid solve of ctx (up to max_solves) into buf (device,
 * FP32, 3 ng^3 per solve: r0 with zeros outside the active box, phi_old,
 * and the converged change phi - phi_old), the training pairs of the net.  */
int sdpm_record(sdpm_ctx* ctx, float* buf_dev, int64_t max_solves);
/* Solves recorded so far, and per solve (up to max) kappa h^2, rms(r0) over
 * the active box and rms(phi_old) over the mesh.                           */
int sdpm_record_info(sdpm_ctx* ctx, int64_t* count, double* kappa_h2, double* rms_r,
                     double* rms_phi, int64_t max);

/* Per-kernel timing (tracing).  enable != 0: every kernel launch made by
 * this context is bracketed by a HIP event pair on the context's stream and
 * charged with its algorithmic bytes (the bytes the method must move: e.g.
 * 2 sizeof(T) per cell for one red-black colour sweep, 72 B per particle for
 * interpolation + kick + drift in FP32 momenta); totals are cleared.  0: off. */
typedef struct sdpm_kernel_stat {
  char name[32];
  int64_t launches;
  double ms;      /* summed event time of the launches, milliseconds */
  double bytes;   /* summed algorithmic bytes                        */
} sdpm_kernel_stat;
int sdpm_profile(sdpm_ctx* ctx, int32_t enable);
/* Like sdpm_profile(ctx, 1) for the kernels named in `names` only (a
 * comma-separated list of the names sdpm_profile_read reports, e.g.
 * "smooth_color"); the other launches get no event pair.  Each event pair
 * costs queue time between launches, so a run timed as a whole brackets only
 * the kernels it needs.  An unknown or empty name: SDPM_EINVAL, profiling
 * left as it was.                                                            */
int sdpm_profile_kernels(sdpm_ctx* ctx, const char* names);
/* Copies min(max, kinds) per-kernel totals to out; *n = number of kinds.
 * Totals cover launches completed by the last synchronising call.          */
int sdpm_profile_read(sdpm_ctx* ctx, sdpm_kernel_stat* out, int32_t max, int32_t* n);

int sdpm_destroy(sdpm_ctx* ctx);

/* Message of the last failure on ctx ("" if none).  Valid until the next
 * call on ctx.  With ctx == NULL: the last failure of sdpm_create.          */
const char* sdpm_last_error(const sdpm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SDPM_H */
