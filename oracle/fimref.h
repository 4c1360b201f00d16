/*
 * fimref.h - FP64 CPU oracle for one fully implicit (FIM) black-oil step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (paper: Sec. 2.1, eqs. (1), (2) and the constraints that
 * follow them, with the black-oil closure stated right after; Sec. 3.2.5 for
 * the four-part Newton iteration; Sec. 3.3.2 for the time-step loop with
 * conditional returns):
 *   backward-Euler, two-point-flux, single-point-upstream residual
 *     R_i,c = (A_i,c(x) - A_i,c(x^n))/dt + sum_faces F_i + sum_perf q_i
 *   in surface units per day, its analytic Jacobian in canonical BSR, and
 *   the Newton/linear iteration that drives R to zero.
 * Where the paper is silent, each function's comment states the reading
 * taken.
 *
 * Units: FIELD (ft, mD, psi, days, rb, stb, Mscf, cP).  Cell id is
 * c = i + nx*(j + ny*k), k = 0 is the top layer.  Unknowns per cell are
 * (P, Sw[, X]) with X = Sg (flag SAT) or Rs (flag UNSAT); equations are
 * (water, oil[, gas]).  One extra block row per well holds its bottom-hole
 * pressure in slot 0; the remaining slots of a well row are identity rows.
 * Vectors are interleaved: entry (row, slot) lives at row*nb + slot.
 * Blocks are row-major: val[(k*nb + eq)*nb + unknown].
 */
#ifndef FIMREF_H
#define FIMREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FR_PROD = 0, FR_INJ_WATER = 1, FR_INJ_GAS = 2 };
enum { FR_BHP = 0, FR_RATE = 1 };
enum { FR_UNSAT = 0, FR_SAT = 1 };

typedef struct {
    int32_t nx, ny, nz;
    const double *dx, *dy, *dz;          /* [nx], [ny], [nz] ft */
    double top;                          /* depth of the top face, ft */
    const double *kx, *ky, *kz, *poro;   /* [N] mD, fraction */
    double cr, pref;                     /* rock compressibility 1/psi, ref P */
    int32_t model;                       /* 2: dead-oil/water, 3: black oil */
    int32_t nrows;                       /* PVT table rows */
    const double *tp, *tbo, *trs, *tmuo, *tbg, *tmug;   /* [nrows] */
    double co_us, cmu_us;                /* undersaturated oil extension */
    double bw_ref, cw, muw, pw_ref;      /* water */
    double rho_w_sc, rho_o_sc, rho_g_sc; /* lb/ft3, lb/ft3, lb/Mscf */
    double swc, sor, sgc, nw, no, ng, krw_max, kro_max, krg_max;
    int32_t nwells;
    const int32_t *wkind, *wctrl;        /* [nwells] */
    const double *wtarget, *wrw, *wskin; /* [nwells] */
    const int32_t *wperf_start;          /* [nwells+1] */
    const int32_t *wperf_cell;           /* [nperf] */
    const double *wperf_wi;              /* [nperf]; <= 0 selects Peaceman */
} fr_input;

/* A caller-supplied solver of J x = rhs (J in the BSR layout of
 * fr_assemble, x returned, *iters its iteration count); 0 on success.  It
 * replaces the solver choice below, e.g. by a sparse direct solve for grids
 * where GMRES with BILU(0) stalls. */
typedef int32_t (*fr_linsolve_fn)(void *ctx, int32_t nrows, int32_t nb, const int32_t *rowptr,
                                  const int32_t *colind, const double *val, const double *rhs,
                                  double *x, int32_t *iters);

typedef struct {
    double tol_cnv, tol_mb, tol_dp, tol_ds, tol_well;
    double ds_max, dp_max, lin_rtol;
    int32_t max_newton, max_lin, restart, max_cuts;
    int32_t dense_max;                   /* dense LU when unknowns <= this */
    int32_t pad;
    fr_linsolve_fn linsolve;             /* NULL: dense LU or GMRES with BILU(0) */
    void *linsolve_ctx;
} fr_options;

#define FR_MAX_SUB 256
typedef struct {
    int32_t newton_iters, linear_iters, cuts, converged, nsub;
    int32_t pad;
    double cnv[3], mb[3];
    double dt_sub[FR_MAX_SUB];           /* accepted sub-step sizes, days */
    double t_assemble, t_linear, t_update;  /* wall seconds per phase */
} fr_report;

typedef struct fr_model fr_model;

/* Setup.  Copies the input; returns NULL and a message via fr_error() on
 * invalid input. */
fr_model *fr_create(const fr_input *in);
void fr_destroy(fr_model *m);
const char *fr_error(void);

int32_t fr_ncells(const fr_model *m);
int32_t fr_nb(const fr_model *m);
int32_t fr_nwells(const fr_model *m);
int32_t fr_nperf(const fr_model *m);
int32_t fr_nnzb(const fr_model *m);
int32_t fr_nprops(const fr_model *m);

/* Static data: cell volume (ft3), centre depth (ft), reference pore volume
 * (rb), transmissibility of the face to the +x/+y/+z neighbour (0 at the
 * outer boundary), per-perforation well index. */
void fr_static(const fr_model *m, double *vol, double *depth, double *pvref,
               double *tx, double *ty, double *tz, double *wi);

/* Canonical BSR pattern of the Jacobian: rowptr[N+W+1], colind[nnzb]. */
void fr_pattern(const fr_model *m, int32_t *rowptr, int32_t *colind);

/* Per-cell property record, structure-of-arrays out[q*N + c].  With
 * np = nb phases (water, oil[, gas]) and a "group" meaning one value
 * followed by its nb derivatives (d/dP, d/dSw[, d/dX]):
 *   np groups   Lam_j  = kr_j * b_j / mu_j
 *   1  group    Lam_og = Rs * Lam_o                 (nb == 3 only)
 *   1  group    lam_t  = sum_j kr_j / mu_j
 *   np groups   gam_j  = rho_j / 144                (psi/ft)
 *   nb groups   A_i    = accumulation of component i (surface units)
 *   np values   b_j    = 1/B_j
 *   1  value    PV     = pore volume at P (rb)
 */
void fr_props(const fr_model *m, const double *P, const double *Sw, const double *X,
              const int8_t *flag, double *out);

/* Accumulation A[c*nb + i] of every component at a state. */
void fr_accum(const fr_model *m, const double *P, const double *Sw, const double *X,
              const int8_t *flag, double *A);

/* Residual R[(N+W)*nb] and (if val != NULL) the analytic Jacobian values in
 * the canonical pattern, at state (P, Sw, X, flag, pbhp) with accumulation
 * at the start of the step Aold[N*nb]. */
void fr_assemble(const fr_model *m, const double *P, const double *Sw, const double *X,
                 const int8_t *flag, const double *pbhp, const double *Aold, double dt,
                 double *R, double *val);

/* Surface well rates q[w*3 + i] (production positive) at a state. */
void fr_well_rates(const fr_model *m, const double *P, const double *Sw, const double *X,
                   const int8_t *flag, const double *pbhp, double *q);

/* Convergence measures at a residual: cnv[3], mb[3] (a reading: the paper
 * defines no norm). */
void fr_conv(const fr_model *m, const double *P, const double *Sw, const double *X,
             const int8_t *flag, const double *R, double dt, double *cnv, double *mb);

/* Linear algebra on a canonical BSR matrix of nrows block rows. */
void fr_bsr_spmv(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const double *x, double *y);
int  fr_bj_setup(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                 const double *val, double *dinv);
void fr_bj_apply(int32_t nrows, int32_t nb, const double *dinv, const double *x, double *y);
int  fr_bilu0_factor(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                     const double *val, double *lu);
void fr_bilu0_solve(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                    const double *lu, const double *b, double *x);
/* Dense LU with partial pivoting, A is n x n row-major (overwritten). */
int  fr_dense_solve(int32_t n, double *A, double *b);
/* Right-preconditioned restarted GMRES with a natural-order BILU(0)
 * preconditioner.  Returns 0 when the true relative residual <= rtol. */
int  fr_gmres_bilu0(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                    const double *val, const double *b, double *x, double rtol,
                    int32_t restart, int32_t max_iter, int32_t *iters, double *relres);

/* One time step of length dt days with deterministic halving cuts.  The
 * state arrays are advanced in place; on failure they hold the step-start
 * state.  Returns 0 on success, 1 when not converged after max_cuts. */
int fr_step(const fr_model *m, double *P, double *Sw, double *X, int8_t *flag,
            double *pbhp, double dt, const fr_options *opt, fr_report *rep);

#ifdef __cplusplus
}
#endif
#endif
