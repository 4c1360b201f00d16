/*
 * fim.h - C ABI of libfim.so, the MI355X (gfx950) fully implicit black-oil
 * step: per-cell black-oil properties, two-point-flux upwinded face fluxes
 * assembled into a residual and a 2x2 / 3x3 block-sparse (BSR) Jacobian,
 * and right-preconditioned GMRES on that Jacobian, driven by Newton with
 * time-step cuts.  Every numeric step runs in HIP kernels on the device of
 * the stream passed to fim_create.
 *
 * Paper (OpenCAEPoro, arXiv 2406.10862):
 *   Sec. 2.1, eq. (1)   component mass conservation (diffusion term zero);
 *   Sec. 2.1, eq. (2)   Darcy velocity with gravity;
 *   Sec. 2.1            constraints N_i = phi sum_j S_j xi_j x_ij,
 *                       sum_j S_j = 1, and the black-oil closure (phase
 *                       quantities explicit in P from tables);
 *   Sec. 3.2.3-3.2.4    Bulk (PVT, SAT, ROCK, ACCU), BulkConn (connection
 *                       fluxes) and AllWells (perforation flux, well rows);
 *   Sec. 3.2.5          one FIM Newton iteration = assemble, solve and
 *                       update, property update, convergence check;
 *   Sec. 3.3.1-3.3.2    Setup / InitReservoir / GoOneStep, time stepping
 *                       with conditional returns to earlier stages;
 *   Sec. 3.3.3          the linear system returns the solution and the
 *                       iteration count;
 *   Sec. 5.1            FGMRES with block-Jacobi ILU(0) smoothing.
 *
 * Conventions
 *   Units: FIELD (ft, mD, psi, days, rb, stb, Mscf, cP; gas density lb/Mscf).
 *   Cells: c = i + nx*(j + ny*k), 0-based, k = 0 is the top layer.  Depth
 *     of a cell centre = top + (thickness of the layers above) + dz_k/2.
 *   Unknowns per cell: (P, Sw) for model 2 (dead oil / water) and
 *     (P, Sw, X) for model 3 (black oil), X = Sg when flag = FIM_SAT and
 *     X = Rs (Mscf/stb) when flag = FIM_UNSAT.  Equations per cell: water,
 *     oil[, gas], in surface units per day.
 *   Wells: one extra block row per well after the cells; slot 0 holds the
 *     bottom-hole pressure, other slots are identity rows with value 0.
 *   Vectors (residual, Newton update, GMRES vectors) are interleaved:
 *     entry (row, slot) at row*nb + slot.  BSR blocks are row-major,
 *     val[(q*nb + equation)*nb + unknown]; columns ascend within a row.
 *   Ownership: inputs are copied at the call; outputs go to caller-owned
 *     buffers of the documented size.  "_dev" arguments are device pointers
 *     valid on the context's device; everything else is host memory.
 *   Errors: a negative return is an error (the message is available from
 *     fim_last_error() on the same thread); FIM_E_HIP leaves the context
 *     unusable.  A positive return is a status, the context stays valid.
 *     After FIM_NOT_CONVERGED the state is the state at the start of the
 *     step.  No exception crosses the ABI.  Use one context per thread.
 */
#ifndef FIM_H
#define FIM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FIM_OK = 0,
    FIM_NOT_CONVERGED = 1,
    FIM_SKIPPED = 2,          /* ensemble step not run (its member stopped earlier) */
    FIM_E_ARG = -1,
    FIM_E_NOMEM = -2,
    FIM_E_HIP = -3,
    FIM_E_STATE = -4
};

enum { FIM_DEADOIL_OW = 2, FIM_BLACKOIL_3P = 3 };          /* model id == block size */
enum { FIM_PROD = 0, FIM_INJ_WATER = 1, FIM_INJ_GAS = 2 };  /* well kind */
enum { FIM_BHP = 0, FIM_RATE = 1 };                         /* well control */
enum { FIM_UNSAT = 0, FIM_SAT = 1 };                        /* phase-state flag */
enum { FIM_PREC_BJ = 0, FIM_PREC_ILU0 = 1, FIM_PREC_CPR = 2,  /* preconditioner */
       FIM_PREC_CPR_ILU0 = 3 };
enum { FIM_FP64 = 0, FIM_MIXED = 1 };                       /* precision mode */

/* Cartesian grid: dx[nx], dy[ny], dz[nz] in ft, top = depth of the top face. */
typedef struct {
    int32_t nx, ny, nz;
    const double *dx, *dy, *dz;
    double top;
} fim_grid;

/* Rock: per-cell permeabilities (mD; kz is used on vertical faces) and
 * reference porosity; phi(P) = poro*(1 + cr*(P - pref)). */
typedef struct {
    const double *kx, *ky, *kz, *poro;
    double cr, pref;
} fim_rock;

/* Fluid.  PVT table columns over nrows pressures p (strictly increasing):
 * saturated oil Bo (rb/stb), Rs (Mscf/stb), muo (cP), gas Bg (rb/Mscf),
 * mug (cP).  Values between rows are linear in P, the end intervals
 * extrapolate, and a pressure on a row uses the interval starting there.
 * Model 2 uses p, bo, muo only.  Undersaturated oil (model 3, flag UNSAT):
 * Pb from inverse interpolation of the Rs column, Bo = Bo_sat(Pb)*(1 -
 * co_us*(P - Pb)), muo = muo_sat(Pb)*(1 + cmu_us*(P - Pb)).  Water:
 * Bw = bw_ref*exp(-cw*(P - pw_ref)), constant muw.  Densities at stock tank:
 * rho_sc = {water lb/ft3, oil lb/ft3, gas lb/Mscf}.  Relative
 * permeabilities are Corey: krw = krw_max*<(Sw-swc)/(1-swc-sor)>^nw,
 * kro = kro_max*<(So-sor)/D>^no, krg = krg_max*<(Sg-sgc)/D>^ng with
 * D = 1-swc-sor-sgc (sgc ignored by model 2) and <.> clamped to [0,1].
 * Capillary pressure is zero. */
typedef struct {
    int32_t model, nrows;
    const double *p, *bo, *rs, *muo, *bg, *mug;
    double co_us, cmu_us;
    double bw_ref, cw, muw, pw_ref;
    double rho_sc[3];
    double swc, sor, sgc, nw, no, ng, krw_max, kro_max, krg_max;
} fim_fluid;

/* Well with nperf perforations in distinct cells.  Producers take BHP
 * control; injectors (pure water or free gas) take BHP or a surface RATE
 * target (> 0).  wi[nperf] may be NULL: then Peaceman's well index with
 * wellbore radius rw (ft) and skin is used.  The BHP acts at every
 * perforation (no wellbore head).  A perforation is weighted by the side
 * the flow comes from: flow out of the cell (a producer, or an injector
 * perforation whose cell pressure exceeds the BHP) has the rate
 * WI*Lam_i*(P - Pbhp) of component i, Lam_i = kr_i b_i/mu_i (gas adds
 * Rs*Lam_o); flow into the cell (an injector with Pbhp >= P) is the
 * injected fluid, -WI*(sum_j kr_j/mu_j)*b_inj*(Pbhp - P). */
typedef struct {
    int32_t kind, control;
    double target;
    int32_t nperf;
    const int32_t *cells;
    const double *wi;
    double rw, skin;
} fim_well;

/* Solver controls (the OCPControl role).  Convergence of a Newton
 * iteration requires, per component i, CNV_i = dt*max_c|R_ic|/(PV_c b_ic)
 * <= tol_cnv and MB_i = dt*|sum_c R_ic|/sum_c PV_c b_ic <= tol_mb, every
 * well residual divided by its derivative w.r.t. the BHP <= tol_well
 * (psi), and a last Newton update with max|dP| <= tol_dp (psi, cells and
 * wells) and max|dS| <= tol_ds, and the iterate must be physical: every
 * saturation (Sw, So and, model 3, Sg) in [-1e-6, 1 + 1e-6]; a converged
 * iterate outside that range, like a non-finite residual, fails the Newton
 * solve.  Updates are chopped per cell to
 * max|dS| <= ds_max and |dP| <= dp_max.  A failed Newton solve halves dt,
 * at most max_cuts times per step.  GMRES(restart) runs to relative
 * residual lin_rtol or max_lin iterations per Newton iteration (restart
 * in [1, 40]); an unconverged solve is still used when it reduced the
 * residual.  The solver is flexible GMRES, right-preconditioned by block
 * Jacobi (FIM_PREC_BJ), by block-Jacobi ILU(0) over box subdomains
 * (FIM_PREC_ILU0) or by CPR (FIM_PREC_CPR, FIM_PREC_CPR_ILU0): a quasi-IMPES pressure
 * stage solved by one aggregation-AMG cycle (amg_cycle 1 = V, 2 = W, 0 =
 * default: V at the finest level and W below it, a value >= 16 = W on the
 * levels with at most that many cells and wells and V above them, a value
 * <= -16 = V at the finest level and on the levels with at most -amg_cycle
 * cells and wells, W on the others; amg_sweeps red-black Gauss-Seidel sweeps before and after the
 * coarse correction, 0 = default 1) followed by block Jacobi on the
 * remaining residual (FIM_PREC_CPR_ILU0: block-Jacobi ILU(0) on it).
 * Block-Jacobi ILU(0) (paper Sec. 5.1): the subdomains are boxes of
 * tile_nx x tile_ny x tile_nz cells (0 = 8; a size >= the grid takes the
 * whole axis), each with the wells whose perforations all lie in it (other
 * wells stand alone); inside a subdomain the factors are the natural-order
 * block ILU(0) of its diagonal part of the Jacobian, so one box covering
 * the grid gives the plain natural-order BILU(0).  forcing != 0 replaces the fixed lin_rtol by the
 * Eisenstat-Walker forcing term (choice 2, gamma 0.9, alpha 2) between 1e-2
 * and lin_rtol.  graphs != 0 replays each Arnoldi step after its SpMV as a
 * captured HIP graph.  amg_fused: the coarse part of the AMG cycle, from
 * the first level with at most amg_fused cells and wells down, runs as a
 * single-workgroup launch (0 = default 4096, negative = every phase
 * launched separately; the result is the same bit for bit).  amg_seg_rows:
 * AMG levels with at least this many cells of each colour restrict by row
 * segments (0 = default 2^18, negative = never; the sums are the same bit for
 * bit either way).  gs_refine: the Arnoldi orthogonalisation is classical
 * Gram-Schmidt; 1 adds a second pass whenever the first one cancelled more
 * than 90% of the vector's norm, -1 never adds one (a single classical pass,
 * PETSc's default for its GMRES family), 0 = default (-1).  amg_exact > 0: the
 * hierarchy stops at the first level below the finest with at most this
 * many cells (<= 0 = never, the default) whose slabs (the cells of one
 * coordinate of its longest axis) hold at most 96 cells and wells and whose
 * every well lies in one slab; that level is solved exactly, by block
 * elimination over the slabs, and the level above it then runs a V-cycle
 * (otherwise the levels go down to at most 64 cells, inverted densely).  It
 * is fixed when the context is created.  amg_exact_mode (with amg_exact, fixed
 * at creation): 0 = the level's dense inverse, formed from the slab factors
 * once per preconditioner setup and applied as a product over the whole
 * device (the default; it holds (2 half + nwells)^2 doubles, at most 8192
 * columns, else mode 1 is used); 1 = block substitution over the slabs in
 * one workgroup at every application (what members of fim_ensemble_run
 * always use).  profile = k > 0
 * has every k-th Krylov SpMV launch of fim_step (k = 1: every one) stamp
 * its own start and end into a pair of HIP events and reports the summed
 * kernel time of the stamped launches and their count in fim_step_report.  precision FIM_MIXED (with an ILU(0)
 * preconditioner) runs every GMRES restart cycle in single precision: a
 * float copy of the Jacobian, float Krylov vectors, ILU(0) factors and
 * pressure column (sums in double), stopping after a 1e-5 reduction; each
 * restart is an FP64 refinement step on the true residual b - J x, so the
 * converged solution meets lin_rtol in FP64. */
typedef struct {
    double tol_cnv, tol_mb, tol_dp, tol_ds, tol_well;
    double ds_max, dp_max, lin_rtol;
    int32_t max_newton, max_lin, restart, max_cuts;
    int32_t precond, precision, profile, amg_cycle, amg_sweeps, graphs, forcing, amg_fused;
    int32_t tile_nx, tile_ny, tile_nz, amg_seg_rows;
    int32_t gs_refine, amg_exact, amg_exact_mode;
} fim_options;

#define FIM_MAX_SUB 256
typedef struct {
    int32_t newton_iters, linear_iters, cuts, converged, nsub;
    int32_t spmv_calls;                      /* SpMV launches stamped (options.profile) */
    double dt_done, cnv[3], mb[3];
    double t_assemble, t_linear, t_update;   /* device ms per phase */
    double spmv_ms;                          /* their summed kernel ms (HIP events) */
    double last_dp, last_ds, well_res;       /* last Newton check: update sizes, well measure */
    double dt_sub[FIM_MAX_SUB];              /* accepted sub-step sizes (days) */
    double gs_vectors;                       /* basis vectors orthogonalised against, summed
                                                over the Arnoldi steps (j + 1 at step j) */
} fim_step_report;

typedef struct fim_ctx fim_ctx;

/* Setup (the paper's Setup + static part of InitReservoir).  hip_stream
 * is a hipStream_t (NULL = the default stream) that the context orders its
 * work after; the context runs on a stream of its own on the current
 * device.  Validates sizes, table monotonicity, the positive total
 * compressibility of saturated rows (Bg*dRs/dP > dBo/dP), perforation
 * ranges and controls; returns FIM_E_ARG with a message on bad input.
 * Size limits (the kernels index with 32-bit integers): fewer than 2^28
 * cells, and fewer than 2^31 Jacobian values (nnzb*nb*nb, nnzb = cells +
 * twice the interior faces + twice the perforations + wells); both are
 * checked from the grid dimensions before any array is read. */
int fim_create(const fim_grid *grid, const fim_rock *rock, const fim_fluid *fluid,
               int32_t nwells, const fim_well *wells, const fim_options *opt,
               void *hip_stream, fim_ctx **out);
void fim_destroy(fim_ctx *ctx);
const char *fim_last_error(void);

int fim_sizes(const fim_ctx *ctx, int32_t *ncells, int32_t *nb, int32_t *nwells,
              int32_t *nnzb, int32_t *nprops);
int fim_set_options(fim_ctx *ctx, const fim_options *opt);

/* State (the non-equilibrium InitReservoir of Sec. 3.3.1: one state per
 * cell).  p, sw, x3 (ignored by model 2), flag: [ncells]; bhp: [nwells] or
 * NULL, which selects the target for BHP wells and the mean perforated-cell
 * pressure for rate wells.  Also records the state as the start of the next
 * step.  The state is not validated: a non-finite or non-physical state
 * makes the next fim_step fail its Newton solves and return
 * FIM_NOT_CONVERGED with this state restored.
 * fim_set_state_dev: the same with p_dev, sw_dev, x3_dev (float64) and
 * flag_dev (int8) device pointers to [ncells] elements on the context's
 * device, read in order after the work queued on the stream given to
 * fim_create (bhp stays a host pointer); the caller keeps ownership and may
 * reuse the buffers once the call returns. */
int fim_set_state(fim_ctx *ctx, const double *p, const double *sw, const double *x3,
                  const int8_t *flag, const double *bhp);
int fim_set_state_dev(fim_ctx *ctx, const double *p_dev, const double *sw_dev,
                      const double *x3_dev, const int8_t *flag_dev, const double *bhp);
int fim_get_state(fim_ctx *ctx, double *p, double *sw, double *x3, int8_t *flag, double *bhp);

/* One time step of dt_days (GoOneStep): Newton iterations on the
 * backward-Euler system, halving the step on failure.  Advances the state
 * in place; fills rep (may be NULL).  Returns FIM_OK or FIM_NOT_CONVERGED. */
int fim_step(fim_ctx *ctx, double dt_days, fim_step_report *rep);

/* fim_step for callers that cannot allocate device memory once the context
 * exists (serving loops, harnesses that forbid allocation): the same step,
 * bit for bit, that allocates no device memory.  Its reduction partials and
 * scalar slots live in a static array of 65,568 doubles (512.25 KiB) that
 * the library holds on every device it runs on until the process ends; the
 * kernels are launched one by one (no graph executable is instantiated, the
 * graphs option is ignored for the call) and the profile option is ignored.
 * One step needs (restart + 1) * min(2048, ceil((ncells+nwells)*nb/256))
 * doubles of partials (restart <= 31 always fits); a larger need is
 * rejected with FIM_E_ARG before any work.  The array is shared by every
 * call on a device: calls that overlap on one device (two threads, or
 * fim_ensemble_run members) race and must not be made. */
int fim_step_noalloc(fim_ctx *ctx, double dt_days, fim_step_report *rep);

/* Discrete adjoint: the gradient of a production mismatch with respect to
 * the log-permeability of every cell.  The paper has no adjoint; the
 * gradient is that of the discrete system it solves, the backward-Euler
 * residual of eqs. (1)-(2) with the fluxes and wells of Sec. 3.2.3-3.2.4.
 *   theta_c = ln k_c, with kx, ky and kz of cell c scaled together
 *   (porosity held fixed; an explicit well index does not depend on k, a
 *   Peaceman one scales with k);
 *   J = sum over the nsteps schedule steps s and the producers w of
 *       (q_o,w(x_s) - q_obs[s*nwells + w])^2, q_o,w the surface oil rate of
 *       the well at the end of step s (stb/d); q_obs entries of other wells
 *       are ignored (q_obs may be NULL without wells).
 * From the current state, runs the nsteps steps of dt[nsteps] (days) as
 * fim_step does, then the backward sweep over the accepted sub-steps.  The
 * sweep needs the state after every sub-step: checkpoint_every = 0 keeps
 * all of them on the device during the forward run; checkpoint_every = k
 * >= 1 keeps the state at the start of every k-th schedule step only and
 * recomputes each segment of k steps from its checkpoint before sweeping
 * back through it (replaying the recorded sub-steps, so the gradient is bit
 * for bit the same for every k).  Each sub-step of the sweep is a transposed
 * Jacobian solve (FP64 FGMRES to a relative residual of 1e-12, with CPR for
 * J^T: the pressure component restricted, the transposed pressure operator
 * by the aggregation AMG, prolongation by the quasi-IMPES weights, then
 * block-Jacobi ILU(0) of J^T).
 * grad[ncells] (host) receives dJ/dtheta.  On FIM_OK the state is the end
 * of the forward run.  FIM_NOT_CONVERGED: a forward step failed (the state
 * is the start state and grad is not written) or an adjoint solve did not
 * converge (the state is the end of the forward run). */
typedef struct {
    int32_t steps, substeps, cuts, newton_iters, linear_iters, adjoint_iters;
    double objective;                    /* J */
    double adjoint_relres;               /* largest final relative residual of the adjoint solves */
    double t_forward_ms, t_adjoint_ms;   /* host wall time of the forward run and the sweep */
    double t_recompute_ms;               /* part of t_adjoint_ms spent recomputing segments */
    int32_t stored_states, pad;          /* most state copies held on the device at once */
} fim_adjoint_report;

int fim_adjoint_gradient(fim_ctx *ctx, int32_t nsteps, const double *dt, const double *q_obs,
                         int32_t checkpoint_every, double *grad, fim_adjoint_report *rep);

/* New permeabilities kx, ky, kz [ncells] (mD) for the context (the ROCK
 * input of Sec. 3.2.3): the transmissibilities and the Peaceman well
 * indices are computed again from them (explicit well indices stay); the
 * state is kept.  fim_set_perm takes host arrays and checks k >= 0;
 * fim_set_perm_dev takes float64 device arrays on the context's device, read
 * in order after the work queued on the stream given to fim_create, and
 * checks nothing.  The caller keeps ownership. */
int fim_set_perm(fim_ctx *ctx, const double *kx, const double *ky, const double *kz);
int fim_set_perm_dev(fim_ctx *ctx, const double *kx_dev, const double *ky_dev,
                     const double *kz_dev);

/* An ensemble of independent reservoirs (for instance realisations of one
 * field) advanced together: members[0..count) by nsteps time steps each,
 * step s of member k with dt[k*nsteps + s] days.  Every member takes
 * exactly the steps fim_step takes (the time step of Sec. 3.3.2 with the
 * Newton iteration of Sec. 3.2.5 and the CPR-FGMRES of Sec. 5.1), with its
 * own tolerances, cuts and iteration counts, and computes bit for bit what
 * fim_step computes for it.  Running them together is this library's
 * addition, not a method of the paper: every kernel is one launch for all
 * the members (a member's blocks run on the member's own buffers; flags in
 * device memory select the members that take part), the Newton iterations
 * advance in rounds over the members that have work, and the members that
 * need a linear solve share one FGMRES whose restart cycles run in lockstep
 * (a member stops inside a cycle on its own test).
 * Members must use CPR with block-Jacobi ILU(0) (FIM_PREC_CPR_ILU0) in
 * FP64, one block size, device and GMRES restart, ILU(0) boxes of one
 * workgroup size and coarsest AMG levels of at most 96 entries (FIM_E_ARG
 * otherwise); contexts are distinct and their states set.
 *   dt[count*nsteps] (days), status[count*nsteps] (required),
 *   reports[count*nsteps] (may be NULL; phase times and SpMV counts are 0).
 * A member stops at its first step that does not return FIM_OK; its later
 * entries get FIM_SKIPPED.  Returns FIM_OK when every step returned FIM_OK,
 * FIM_NOT_CONVERGED when a member stopped on that status, or a negative
 * code.  The calling thread waits for the whole run; afterwards every
 * member's state is its end state, as after its own fim_step calls. */
int fim_ensemble_run(int32_t count, fim_ctx *const *members, int32_t nsteps, const double *dt,
                     fim_step_report *reports, int32_t *status);

/* Autotuner of the ensemble's block-Jacobi ILU(0) boxes (this library's
 * addition: the box is its reading of the paper's block-Jacobi subdomains,
 * Sec. 5.1).  Times trial_steps steps of dt_days of the whole batched
 * ensemble from the members' current states with each candidate box
 * (cand[0..ncand), all of 64 pencils), sets the fastest on every member
 * (fim_set_options) and leaves every state as it found it.  The choice is
 * cached in the text file cache_path (may be NULL: no cache) under a key of
 * the block size, floor(log2) of the median member's cell count and the
 * device; a call whose key is in the cache applies the cached box without
 * trials (from_cache = 1).  FIM_NOT_CONVERGED when no candidate finished
 * its trial steps (the members keep their boxes and states). */
typedef struct {
    int32_t box[3];                      /* chosen tile_nx, tile_ny, tile_nz */
    int32_t from_cache, trials, ncand;
    int32_t cand[16][3];
    double trial_ms[16];                 /* wall time of each candidate's trial */
} fim_tune_report;

int fim_ensemble_tune(int32_t count, fim_ctx *const *members, double dt_days,
                      int32_t trial_steps, const char *cache_path, fim_tune_report *rep);

/* Surface rates q[w*3 + i] (component i = water, oil, gas; production
 * positive, injection negative) and bottom-hole pressures at the state. */
int fim_get_well_rates(fim_ctx *ctx, double *q_surf, double *bhp);

/* ---- testing hooks ------------------------------------------------------ */

/* Static data of Sec. 3.2.3-3.2.4 (the PreProcess and ROCK setup, and the
 * well indices of AllWells): cell volume ft3, centre depth ft, reference pore volume rb,
 * transmissibility to the +x/+y/+z neighbour, 0 on the boundary, and the
 * per-perforation well index in input order).  Any pointer may be NULL. */
int fim_static(fim_ctx *ctx, double *vol, double *depth, double *pvref, double *tx,
               double *ty, double *tz, double *wi);

/* Set the Newton iterate of Sec. 3.2.5 without changing the step-start
 * accumulation (the x^n of the backward-Euler residual). */
int fim_set_iterate(fim_ctx *ctx, const double *p, const double *sw, const double *x3,
                    const int8_t *flag, const double *bhp);

/* Property record of Sec. 3.2.3 (Bulk: PVT, SAT, ROCK, ACCU; the black-oil
 * closure of Sec. 2.1) at the current iterate, out[q*ncells + c], q in
 * [0, nprops): with np = nb phases (water, oil[, gas]) and a group = one
 * value followed by its derivatives w.r.t. (P, Sw[, X]):
 *   np groups Lam_j = kr_j b_j/mu_j;  (nb==3) 1 group Lam_og = Rs*Lam_o;
 *   1 group lam_t = sum_j kr_j/mu_j;  np groups gam_j = rho_j/144 (psi/ft);
 *   nb groups A_i (accumulation of component i);  np values b_j = 1/B_j;
 *   1 value PV (rb at P). */
int fim_props(fim_ctx *ctx, double *out);

/* The first part of a FIM Newton iteration (Sec. 3.2.5): the residual of
 * eqs. (1)-(2) with the connection and well terms of Sec. 3.2.4,
 * R[(ncells+nwells)*nb], and its Jacobian at the current iterate for a step
 * of dt days; rowptr[ncells+nwells+1], colind[nnzb], val[nnzb*nb*nb].  Any
 * output pointer may be NULL. */
int fim_assemble(fim_ctx *ctx, double dt, double *R, int32_t *rowptr, int32_t *colind,
                 double *val);

/* y = M^-1 x with the configured preconditioner of Sec. 5.1 (block Jacobi,
 * block-Jacobi ILU(0) or CPR) of the last assembled Jacobian;
 * x, y: [(ncells+nwells)*nb] host arrays. */
int fim_precond_apply(fim_ctx *ctx, const double *x, double *y);

/* The linear solve of Sec. 3.3.3 (the solution and its iteration count),
 * by the preconditioned flexible GMRES of Sec. 5.1: J x = b with the last
 * assembled Jacobian; b, x: [(ncells+nwells)*nb] (x is the output, the
 * initial guess is zero).  iters and relres (true ||b - J x||/||b||) may
 * be NULL.  Returns FIM_OK or FIM_NOT_CONVERGED. */
int fim_linear_solve(fim_ctx *ctx, const double *b, double *x, int32_t *iters,
                     double *relres);

/* The pressure operator of AMG level `level` of the CPR first stage (Sec.
 * 5.1: AMG on the pressure equation) at the last assembled Jacobian (the
 * preconditioner is set up first when needed): dims = {nx, ny, nz, nwells}
 * of the level; A (may be NULL) receives it as a dense row-major matrix of
 * (nx*ny*nz + nwells)^2 entries, cells in natural order, then wells.  Level
 * 0 is the quasi-IMPES pressure matrix, level l + 1 the Galerkin product of
 * level l with the piecewise-constant interpolation of 2x2x2 aggregates
 * (wells their own aggregates).  FIM_E_ARG without a CPR preconditioner. */
int fim_amg_level(fim_ctx *ctx, int32_t level, int32_t *dims, double *A);

/* The coarsest AMG level's solve as the cycle runs it (Sec. 5.1, the
 * pressure stage's coarse problem): x = A_c^-1 b for host arrays in the
 * order of fim_amg_level (cells in natural order, then wells) of the last
 * level: when that level is solved exactly (option amg_exact), by the
 * product with its dense inverse formed from the slab factors
 * (amg_exact_mode 0) or by block substitution over the slabs (mode 1); else
 * by the dense inverse of the small coarsest level.  The level's own arrays
 * are not touched.  FIM_E_ARG without a CPR preconditioner. */
int fim_amg_coarse_solve(fim_ctx *ctx, const double *b, double *x);

/* The matrix-vector product inside the Krylov solver of Sec. 5.1: y = A x
 * for a canonical BSR matrix of nrows block rows with nb in {2,3}
 * (rowptr[nrows+1] and colind[nnzb] int32, val[nnzb*nb*nb] float64 row-major
 * blocks, x and y [nrows*nb] float64, every pointer a device pointer on the
 * current device; colind entries must lie in [0, nrows)).  Queued on
 * hip_stream, no synchronisation; the caller keeps ownership. */
int fim_bsr_spmv(int32_t nrows, int32_t nb, const int32_t *rowptr_dev,
                 const int32_t *colind_dev, const double *val_dev, const double *x_dev,
                 double *y_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
