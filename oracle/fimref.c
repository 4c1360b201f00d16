/*
 * fimref.c - FP64 CPU oracle for one fully implicit black-oil time step.
 *
 * TEST INFRASTRUCTURE ONLY (see fimref.h).  Plain C, written for clarity:
 * face-by-face scatter, textbook block ILU(0), modified Gram-Schmidt GMRES,
 * dense LU with partial pivoting.  OpenMP is used only on independent
 * per-cell loops and vector operations.
 *
 * Paper anchors (cited by section, no line numbers):
 *   Sec. 2.1 eq. (1)  component conservation, here with zero diffusion;
 *   Sec. 2.1 eq. (2)  Darcy velocity with gravity;
 *   Sec. 2.1 constraints N_i = phi sum_j S_j xi_j x_ij and sum_j S_j = 1;
 *   Sec. 2.1 black-oil closure: phase data explicit in P (tables);
 *   Sec. 3.2.3 Bulk::PVT / SAT / ROCK / ACCU; Sec. 3.2.4 BulkConn fluxes, AllWells;
 *   Sec. 3.2.5 the four parts of one FIM Newton iteration;
 *   Sec. 3.3.2 time stepping with conditional returns (cuts);
 *   Sec. 5.1   FGMRES with block-Jacobi ILU(0) as the iterative solver.
 */
#include "fimref.h"

#include <math.h>
#include <omp.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* FIELD-unit constants */
#define DARCY 0.001127      /* mD*ft -> rb*cP/(day*psi) */
#define FT3_PER_BBL 5.615
#define PSI_PER_LBFT2 144.0

static __thread char g_err[512];
const char *fr_error(void) { return g_err; }

struct fr_model {
    int n, nx, ny, nz, nb, np, nw, nperf, nrows, nnzb;
    double top, cr, pref;
    double *dx, *dy, *dz, *kx, *ky, *kz, *poro;
    double *tp, *tbo, *trs, *tmuo, *tbg, *tmug;
    double co_us, cmu_us, bw_ref, cw, muw, pw_ref;
    double rho_w_sc, rho_o_sc, rho_g_sc;
    double swc, sor, sgc, nw_, no_, ng_, krw_max, kro_max, krg_max;
    int *wkind, *wctrl, *wps, *wpc;
    double *wtarget, *wrw, *wskin, *wi;
    /* static */
    double *vol, *depth, *pvref, *tx, *ty, *tz;
    int *rowptr, *colind;
};

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    if (!p) { fprintf(stderr, "fimref: out of memory\n"); abort(); }
    return p;
}
static double *dup_d(const double *a, int n) {
    double *p = (double *)xcalloc((size_t)n, sizeof(double));
    if (a) memcpy(p, a, sizeof(double) * (size_t)n);
    return p;
}
static int *dup_i(const int32_t *a, int n) {
    int *p = (int *)xcalloc((size_t)n, sizeof(int));
    if (a) for (int i = 0; i < n; ++i) p[i] = a[i];
    return p;
}

int32_t fr_ncells(const fr_model *m) { return m->n; }
int32_t fr_nb(const fr_model *m) { return m->nb; }
int32_t fr_nwells(const fr_model *m) { return m->nw; }
int32_t fr_nperf(const fr_model *m) { return m->nperf; }
int32_t fr_nnzb(const fr_model *m) { return m->nnzb; }
int32_t fr_nprops(const fr_model *m) {
    int nb = m->nb, np = m->np;
    return np * (nb + 1) + (nb == 3 ? nb + 1 : 0) + (nb + 1) + np * (nb + 1) +
           nb * (nb + 1) + np + 1;
}

/* ------------------------------------------------------------------------ */
/* Static data: volumes, depths, pore volumes, TPFA transmissibilities and
 * Peaceman well indices.  Transmissibility is the harmonic combination of
 * the two half-cell conductances, with kv on vertical faces. */

static int cid(const fr_model *m, int i, int j, int k) { return i + m->nx * (j + m->ny * k); }

static double half_trans(double perm, double area, double half_len) {
    return perm * area / half_len;   /* mD*ft */
}

static double face_trans(double k1, double d1, double k2, double d2, double area) {
    /* T = DARCY * A / (d1/k1 + d2/k2), written as a harmonic sum of the two
     * half transmissibilities k*A/d. */
    double t1 = half_trans(k1, area, d1), t2 = half_trans(k2, area, d2);
    if (t1 <= 0.0 || t2 <= 0.0) return 0.0;
    return DARCY / (1.0 / t1 + 1.0 / t2);
}

static double peaceman_wi(double kx, double ky, double dx, double dy, double h,
                          double rw, double skin) {
    double ryx = sqrt(ky / kx), rxy = sqrt(kx / ky);
    double ro = 0.28 * sqrt(ryx * dx * dx + rxy * dy * dy) /
                (pow(ky / kx, 0.25) + pow(kx / ky, 0.25));
    return DARCY * 2.0 * M_PI * sqrt(kx * ky) * h / (log(ro / rw) + skin);
}

static void compute_static(fr_model *m) {
    int n = m->n;
    m->vol = (double *)xcalloc(n, sizeof(double));
    m->depth = (double *)xcalloc(n, sizeof(double));
    m->pvref = (double *)xcalloc(n, sizeof(double));
    m->tx = (double *)xcalloc(n, sizeof(double));
    m->ty = (double *)xcalloc(n, sizeof(double));
    m->tz = (double *)xcalloc(n, sizeof(double));
    for (int k = 0; k < m->nz; ++k) {
        double above = 0.0;
        for (int kk = 0; kk < k; ++kk) above += m->dz[kk];
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                int c = cid(m, i, j, k);
                m->vol[c] = m->dx[i] * m->dy[j] * m->dz[k];
                m->depth[c] = m->top + above + 0.5 * m->dz[k];
                m->pvref[c] = m->vol[c] * m->poro[c] / FT3_PER_BBL;
                if (i + 1 < m->nx) {
                    int d = cid(m, i + 1, j, k);
                    m->tx[c] = face_trans(m->kx[c], 0.5 * m->dx[i], m->kx[d], 0.5 * m->dx[i + 1],
                                          m->dy[j] * m->dz[k]);
                }
                if (j + 1 < m->ny) {
                    int d = cid(m, i, j + 1, k);
                    m->ty[c] = face_trans(m->ky[c], 0.5 * m->dy[j], m->ky[d], 0.5 * m->dy[j + 1],
                                          m->dx[i] * m->dz[k]);
                }
                if (k + 1 < m->nz) {
                    int d = cid(m, i, j, k + 1);
                    m->tz[c] = face_trans(m->kz[c], 0.5 * m->dz[k], m->kz[d], 0.5 * m->dz[k + 1],
                                          m->dx[i] * m->dy[j]);
                }
            }
    }
    for (int w = 0; w < m->nw; ++w)
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) {
            if (m->wi[p] > 0.0) continue;
            int c = m->wpc[p];
            int i = c % m->nx, j = (c / m->nx) % m->ny, k = c / (m->nx * m->ny);
            m->wi[p] = peaceman_wi(m->kx[c], m->ky[c], m->dx[i], m->dy[j], m->dz[k], m->wrw[w],
                                   m->wskin[w]);
        }
}

void fr_static(const fr_model *m, double *vol, double *depth, double *pvref, double *tx,
               double *ty, double *tz, double *wi) {
    size_t b = sizeof(double) * (size_t)m->n;
    if (vol) memcpy(vol, m->vol, b);
    if (depth) memcpy(depth, m->depth, b);
    if (pvref) memcpy(pvref, m->pvref, b);
    if (tx) memcpy(tx, m->tx, b);
    if (ty) memcpy(ty, m->ty, b);
    if (tz) memcpy(tz, m->tz, b);
    if (wi) memcpy(wi, m->wi, sizeof(double) * (size_t)m->nperf);
}

/* ------------------------------------------------------------------------ */
/* Sparsity pattern: natural cell order, well rows after the cells (Sec.
 * 3.4.1 orders interior cells by ascending global index; the well rows "w"
 * of the parallel-strategy figure are appended).  Each row lists its
 * columns in ascending order. */

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static void build_pattern(fr_model *m) {
    int n = m->n, nw = m->nw, nrow = n + nw;
    int *cnt = (int *)xcalloc(nrow, sizeof(int));
    /* count */
    for (int c = 0; c < n; ++c) {
        int i = c % m->nx, j = (c / m->nx) % m->ny, k = c / (m->nx * m->ny);
        cnt[c] = 1 + (i > 0) + (i + 1 < m->nx) + (j > 0) + (j + 1 < m->ny) + (k > 0) +
                 (k + 1 < m->nz);
    }
    for (int w = 0; w < nw; ++w) {
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) cnt[m->wpc[p]] += 1;
        cnt[n + w] = (m->wps[w + 1] - m->wps[w]) + 1;
    }
    m->rowptr = (int *)xcalloc(nrow + 1, sizeof(int));
    for (int r = 0; r < nrow; ++r) m->rowptr[r + 1] = m->rowptr[r] + cnt[r];
    m->nnzb = m->rowptr[nrow];
    m->colind = (int *)xcalloc(m->nnzb, sizeof(int));
    int *fill = (int *)xcalloc(nrow, sizeof(int));
    int nxy = m->nx * m->ny;
    for (int c = 0; c < n; ++c) {
        int i = c % m->nx, j = (c / m->nx) % m->ny, k = c / nxy;
        int *dst = m->colind + m->rowptr[c];
        int q = 0;
        dst[q++] = c;
        if (i > 0) dst[q++] = c - 1;
        if (i + 1 < m->nx) dst[q++] = c + 1;
        if (j > 0) dst[q++] = c - m->nx;
        if (j + 1 < m->ny) dst[q++] = c + m->nx;
        if (k > 0) dst[q++] = c - nxy;
        if (k + 1 < m->nz) dst[q++] = c + nxy;
        fill[c] = q;
    }
    for (int w = 0; w < nw; ++w) {
        int *dst = m->colind + m->rowptr[n + w];
        int q = 0;
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) {
            int c = m->wpc[p];
            m->colind[m->rowptr[c] + fill[c]++] = n + w;
            dst[q++] = c;
        }
        dst[q++] = n + w;
        fill[n + w] = q;
    }
    for (int r = 0; r < nrow; ++r)
        qsort(m->colind + m->rowptr[r], (size_t)cnt[r], sizeof(int), cmp_int);
    free(cnt);
    free(fill);
}

void fr_pattern(const fr_model *m, int32_t *rowptr, int32_t *colind) {
    for (int r = 0; r <= m->n + m->nw; ++r) rowptr[r] = m->rowptr[r];
    for (int q = 0; q < m->nnzb; ++q) colind[q] = m->colind[q];
}

/* position of block (row, col) in the value array */
static int blk(const fr_model *m, int row, int col) {
    for (int q = m->rowptr[row]; q < m->rowptr[row + 1]; ++q)
        if (m->colind[q] == col) return q;
    fprintf(stderr, "fimref: block (%d,%d) not in pattern\n", row, col);
    abort();
}

/* ------------------------------------------------------------------------ */

fr_model *fr_create(const fr_input *in) {
    g_err[0] = 0;
    if (!in || in->nx < 1 || in->ny < 1 || in->nz < 1) {
        snprintf(g_err, sizeof g_err, "bad grid dimensions");
        return NULL;
    }
    if (in->model != 2 && in->model != 3) {
        snprintf(g_err, sizeof g_err, "model must be 2 or 3");
        return NULL;
    }
    if (in->nrows < 2) {
        snprintf(g_err, sizeof g_err, "PVT table needs >= 2 rows");
        return NULL;
    }
    for (int r = 0; r + 1 < in->nrows; ++r)
        if (!(in->tp[r + 1] > in->tp[r])) {
            snprintf(g_err, sizeof g_err, "PVT pressure column not increasing");
            return NULL;
        }
    if (in->model == 3)
        for (int r = 0; r + 1 < in->nrows; ++r)
            if (!(in->trs[r + 1] > in->trs[r])) {
                snprintf(g_err, sizeof g_err, "Rs column not increasing");
                return NULL;
            }
    fr_model *m = (fr_model *)xcalloc(1, sizeof(fr_model));
    m->nx = in->nx; m->ny = in->ny; m->nz = in->nz;
    m->n = in->nx * in->ny * in->nz;
    m->nb = in->model; m->np = in->model;
    m->top = in->top; m->cr = in->cr; m->pref = in->pref;
    m->dx = dup_d(in->dx, in->nx); m->dy = dup_d(in->dy, in->ny); m->dz = dup_d(in->dz, in->nz);
    m->kx = dup_d(in->kx, m->n); m->ky = dup_d(in->ky, m->n); m->kz = dup_d(in->kz, m->n);
    m->poro = dup_d(in->poro, m->n);
    m->nrows = in->nrows;
    m->tp = dup_d(in->tp, in->nrows); m->tbo = dup_d(in->tbo, in->nrows);
    m->trs = dup_d(in->trs, in->nrows); m->tmuo = dup_d(in->tmuo, in->nrows);
    m->tbg = dup_d(in->tbg, in->nrows); m->tmug = dup_d(in->tmug, in->nrows);
    m->co_us = in->co_us; m->cmu_us = in->cmu_us;
    m->bw_ref = in->bw_ref; m->cw = in->cw; m->muw = in->muw; m->pw_ref = in->pw_ref;
    m->rho_w_sc = in->rho_w_sc; m->rho_o_sc = in->rho_o_sc; m->rho_g_sc = in->rho_g_sc;
    m->swc = in->swc; m->sor = in->sor; m->sgc = in->sgc;
    m->nw_ = in->nw; m->no_ = in->no; m->ng_ = in->ng;
    m->krw_max = in->krw_max; m->kro_max = in->kro_max; m->krg_max = in->krg_max;
    m->nw = in->nwells;
    m->wkind = dup_i(in->wkind, m->nw); m->wctrl = dup_i(in->wctrl, m->nw);
    m->wtarget = dup_d(in->wtarget, m->nw); m->wrw = dup_d(in->wrw, m->nw);
    m->wskin = dup_d(in->wskin, m->nw);
    m->wps = dup_i(in->wperf_start, m->nw + 1);
    m->nperf = m->nw ? m->wps[m->nw] : 0;
    m->wpc = dup_i(in->wperf_cell, m->nperf);
    m->wi = dup_d(in->wperf_wi, m->nperf);
    for (int w = 0; w < m->nw; ++w) {
        if (m->wkind[w] == FR_INJ_GAS && m->nb != 3) {
            snprintf(g_err, sizeof g_err, "gas injector needs the three-phase model");
            fr_destroy(m);
            return NULL;
        }
        if (m->wctrl[w] == FR_RATE && m->wkind[w] == FR_PROD) {
            snprintf(g_err, sizeof g_err, "rate-controlled producers are not supported");
            fr_destroy(m);
            return NULL;
        }
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) {
            if (m->wpc[p] < 0 || m->wpc[p] >= m->n) {
                snprintf(g_err, sizeof g_err, "perforation cell out of range");
                fr_destroy(m);
                return NULL;
            }
            for (int p2 = m->wps[w]; p2 < p; ++p2)
                if (m->wpc[p2] == m->wpc[p]) {
                    snprintf(g_err, sizeof g_err, "duplicate perforation cell");
                    fr_destroy(m);
                    return NULL;
                }
        }
    }
    compute_static(m);
    build_pattern(m);
    return m;
}

void fr_destroy(fr_model *m) {
    if (!m) return;
    double *d[] = {m->dx, m->dy, m->dz, m->kx, m->ky, m->kz, m->poro, m->tp, m->tbo,
                   m->trs, m->tmuo, m->tbg, m->tmug, m->wtarget, m->wrw, m->wskin, m->wi,
                   m->vol, m->depth, m->pvref, m->tx, m->ty, m->tz};
    for (size_t i = 0; i < sizeof d / sizeof d[0]; ++i) free(d[i]);
    free(m->wkind); free(m->wctrl); free(m->wps); free(m->wpc);
    free(m->rowptr); free(m->colind);
    free(m);
}

/* ------------------------------------------------------------------------ */
/* Cell properties (Bulk::PVT, SAT, ROCK, ACCU) with derivatives with respect
 * to the cell's unknowns u = 0:P, 1:Sw, 2:X. */

typedef struct {
    double lam[3], dlam[3][3];     /* kr_j b_j / mu_j          */
    double lamog, dlamog[3];       /* Rs * lam_o               */
    double lt, dlt[3];             /* sum_j kr_j / mu_j        */
    double gam[3], dgam[3][3];     /* rho_j / 144              */
    double acc[3], dacc[3][3];     /* component accumulations  */
    double b[3], dbP[3];           /* 1/B_j and d(1/B_j)/dP    */
    double pv;
} cellprops;

/* interval i in [0, nrows-2] with t[i] <= v < t[i+1]; clamped at both ends,
 * so values outside the table extrapolate the end intervals (the paper gives no interpolation rule: this is a reading) */
static int tab_interval(const double *t, int nrows, double v) {
    int i = 0;
    while (i < nrows - 2 && t[i + 1] <= v) ++i;
    return i;
}

static void tab_eval(const double *t, const double *y, int i, double v, double *val,
                     double *slope) {
    double s = (y[i + 1] - y[i]) / (t[i + 1] - t[i]);
    *slope = s;
    *val = y[i] + s * (v - t[i]);
}

/* Corey relative permeability kr = krmax * <(s_num)/denom>^n, clamped to
 * [0,1]; the derivative is taken on the open interval only. */
static void corey(double s_num, double denom, double krmax, double n, double *kr,
                  double *dkr) {
    double s = s_num / denom;
    if (s <= 0.0) { *kr = 0.0; *dkr = 0.0; }
    else if (s >= 1.0) { *kr = krmax; *dkr = 0.0; }
    else { *kr = krmax * pow(s, n); *dkr = krmax * n * pow(s, n - 1.0) / denom; }
}

static void eval_cell(const fr_model *m, int c, double P, double Sw, double X, int flag,
                      cellprops *cp) {
    memset(cp, 0, sizeof *cp);
    int nb = m->nb;
    /* water: B_w = B_w,ref exp(-c_w (P - P_ref,w)), constant viscosity */
    double bw = exp(m->cw * (P - m->pw_ref)) / m->bw_ref;
    double dbw = m->cw * bw;
    double muw = m->muw;

    /* oil and gas PVT */
    double Rs = 0, dRsP = 0, dRsX = 0;
    double Bo, dBoP, dBoX = 0, muo, dmuoP, dmuoX = 0;
    double Bg = 1, dBgP = 0, mug = 1, dmugP = 0;
    double Sg = 0, dSgX = 0;
    if (nb == 2) {
        int i = tab_interval(m->tp, m->nrows, P);
        tab_eval(m->tp, m->tbo, i, P, &Bo, &dBoP);
        tab_eval(m->tp, m->tmuo, i, P, &muo, &dmuoP);
    } else if (flag == FR_SAT) {
        int i = tab_interval(m->tp, m->nrows, P);
        tab_eval(m->tp, m->trs, i, P, &Rs, &dRsP);
        tab_eval(m->tp, m->tbo, i, P, &Bo, &dBoP);
        tab_eval(m->tp, m->tmuo, i, P, &muo, &dmuoP);
        Sg = X; dSgX = 1.0;
    } else {
        /* undersaturated: bubble point from the inverse of the Rs column,
         * saturated values at Pb on the same interval, linear extension in
         * P - Pb (a reading: the paper leaves undersaturated oil open) */
        Rs = X; dRsX = 1.0;
        int i = tab_interval(m->trs, m->nrows, Rs);
        double dPb = (m->tp[i + 1] - m->tp[i]) / (m->trs[i + 1] - m->trs[i]);
        double Pb = m->tp[i] + (Rs - m->trs[i]) * dPb;
        double Bob, sBo, mub, smu;
        tab_eval(m->tp, m->tbo, i, Pb, &Bob, &sBo);
        tab_eval(m->tp, m->tmuo, i, Pb, &mub, &smu);
        double co = m->co_us, cm = m->cmu_us;
        Bo = Bob * (1.0 - co * (P - Pb));
        dBoP = -Bob * co;
        dBoX = (sBo * (1.0 - co * (P - Pb)) + Bob * co) * dPb;
        muo = mub * (1.0 + cm * (P - Pb));
        dmuoP = mub * cm;
        dmuoX = (smu * (1.0 + cm * (P - Pb)) - mub * cm) * dPb;
    }
    if (nb == 3) {
        int i = tab_interval(m->tp, m->nrows, P);
        tab_eval(m->tp, m->tbg, i, P, &Bg, &dBgP);
        tab_eval(m->tp, m->tmug, i, P, &mug, &dmugP);
    }
    double bo = 1.0 / Bo, dboP = -dBoP / (Bo * Bo), dboX = -dBoX / (Bo * Bo);
    double bg = 1.0 / Bg, dbgP = -dBgP / (Bg * Bg);

    /* densities and gravity gradients */
    double num = FT3_PER_BBL * m->rho_o_sc + Rs * m->rho_g_sc;
    double rhow = m->rho_w_sc * bw, drhowP = m->rho_w_sc * dbw;
    double rhoo = num * bo / FT3_PER_BBL;
    double drhooP = (dRsP * m->rho_g_sc * bo + num * dboP) / FT3_PER_BBL;
    double drhooX = (dRsX * m->rho_g_sc * bo + num * dboX) / FT3_PER_BBL;
    double rhog = m->rho_g_sc * bg / FT3_PER_BBL, drhogP = m->rho_g_sc * dbgP / FT3_PER_BBL;
    cp->gam[0] = rhow / PSI_PER_LBFT2;
    cp->dgam[0][0] = drhowP / PSI_PER_LBFT2;
    cp->gam[1] = rhoo / PSI_PER_LBFT2;
    cp->dgam[1][0] = drhooP / PSI_PER_LBFT2;
    if (nb == 3) {
        cp->dgam[1][2] = drhooX / PSI_PER_LBFT2;
        cp->gam[2] = rhog / PSI_PER_LBFT2;
        cp->dgam[2][0] = drhogP / PSI_PER_LBFT2;
    }

    /* saturations and relative permeabilities (simple Corey; the paper names no three-phase model) */
    double So = 1.0 - Sw - Sg, dSoX = -dSgX;
    double krw, dkrw, kro, dkro, krg = 0, dkrg = 0;
    corey(Sw - m->swc, 1.0 - m->swc - m->sor, m->krw_max, m->nw_, &krw, &dkrw);
    double dgo = 1.0 - m->swc - m->sor - (nb == 3 ? m->sgc : 0.0);
    corey(So - m->sor, dgo, m->kro_max, m->no_, &kro, &dkro);
    if (nb == 3) corey(Sg - m->sgc, dgo, m->krg_max, m->ng_, &krg, &dkrg);
    /* chain rule to the unknowns */
    double dkroSw = -dkro, dkroX = dkro * dSoX, dkrgX = dkrg * dSgX;

    /* Lam_j = kr_j b_j / mu_j */
    cp->lam[0] = krw * bw / muw;
    cp->dlam[0][0] = krw * dbw / muw;
    cp->dlam[0][1] = dkrw * bw / muw;
    double bmo = bo / muo;
    double dbmoP = dboP / muo - bo * dmuoP / (muo * muo);
    double dbmoX = dboX / muo - bo * dmuoX / (muo * muo);
    cp->lam[1] = kro * bmo;
    cp->dlam[1][0] = kro * dbmoP;
    cp->dlam[1][1] = dkroSw * bmo;
    if (nb == 3) {
        cp->dlam[1][2] = dkroX * bmo + kro * dbmoX;
        double bmg = bg / mug, dbmgP = dbgP / mug - bg * dmugP / (mug * mug);
        cp->lam[2] = krg * bmg;
        cp->dlam[2][0] = krg * dbmgP;
        cp->dlam[2][2] = dkrgX * bmg;
        cp->lamog = Rs * cp->lam[1];
        cp->dlamog[0] = dRsP * cp->lam[1] + Rs * cp->dlam[1][0];
        cp->dlamog[1] = Rs * cp->dlam[1][1];
        cp->dlamog[2] = dRsX * cp->lam[1] + Rs * cp->dlam[1][2];
    }
    /* total mobility (injector perforations) */
    cp->lt = krw / muw + kro / muo + (nb == 3 ? krg / mug : 0.0);
    cp->dlt[0] = -kro * dmuoP / (muo * muo) - (nb == 3 ? krg * dmugP / (mug * mug) : 0.0);
    cp->dlt[1] = dkrw / muw + dkroSw / muo;
    if (nb == 3) cp->dlt[2] = dkroX / muo - kro * dmuoX / (muo * muo) + dkrgX / mug;

    /* pore volume and accumulations, N_i = PV * sum_j S_j b_j x_ij */
    double pv = m->pvref[c] * (1.0 + m->cr * (P - m->pref));
    double dpv = m->pvref[c] * m->cr;
    cp->pv = pv;
    cp->b[0] = bw; cp->b[1] = bo; cp->b[2] = (nb == 3) ? bg : 0.0;
    cp->dbP[0] = dbw; cp->dbP[1] = dboP; cp->dbP[2] = (nb == 3) ? dbgP : 0.0;
    cp->acc[0] = pv * bw * Sw;
    cp->dacc[0][0] = dpv * bw * Sw + pv * dbw * Sw;
    cp->dacc[0][1] = pv * bw;
    cp->acc[1] = pv * bo * So;
    cp->dacc[1][0] = dpv * bo * So + pv * dboP * So;
    cp->dacc[1][1] = -pv * bo;
    if (nb == 3) {
        cp->dacc[1][2] = pv * (dboX * So + bo * dSoX);
        double G = bg * Sg + Rs * bo * So;
        double dGP = dbgP * Sg + (dRsP * bo + Rs * dboP) * So;
        double dGSw = -Rs * bo;
        double dGX = bg * dSgX + (dRsX * bo + Rs * dboX) * So + Rs * bo * dSoX;
        cp->acc[2] = pv * G;
        cp->dacc[2][0] = dpv * G + pv * dGP;
        cp->dacc[2][1] = pv * dGSw;
        cp->dacc[2][2] = pv * dGX;
    }
}

void fr_props(const fr_model *m, const double *P, const double *Sw, const double *X,
              const int8_t *flag, double *out) {
    int n = m->n, nb = m->nb, np = m->np;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < n; ++c) {
        cellprops cp;
        eval_cell(m, c, P[c], Sw[c], X ? X[c] : 0.0, flag ? flag[c] : 0, &cp);
        int q = 0;
#define PUT(v) out[(size_t)(q++) * n + c] = (v)
        for (int j = 0; j < np; ++j) {
            PUT(cp.lam[j]);
            for (int u = 0; u < nb; ++u) PUT(cp.dlam[j][u]);
        }
        if (nb == 3) {
            PUT(cp.lamog);
            for (int u = 0; u < nb; ++u) PUT(cp.dlamog[u]);
        }
        PUT(cp.lt);
        for (int u = 0; u < nb; ++u) PUT(cp.dlt[u]);
        for (int j = 0; j < np; ++j) {
            PUT(cp.gam[j]);
            for (int u = 0; u < nb; ++u) PUT(cp.dgam[j][u]);
        }
        for (int i = 0; i < nb; ++i) {
            PUT(cp.acc[i]);
            for (int u = 0; u < nb; ++u) PUT(cp.dacc[i][u]);
        }
        for (int j = 0; j < np; ++j) PUT(cp.b[j]);
        PUT(cp.pv);
#undef PUT
    }
}

void fr_accum(const fr_model *m, const double *P, const double *Sw, const double *X,
              const int8_t *flag, double *A) {
    int nb = m->nb;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m->n; ++c) {
        cellprops cp;
        eval_cell(m, c, P[c], Sw[c], X ? X[c] : 0.0, flag ? flag[c] : 0, &cp);
        for (int i = 0; i < nb; ++i) A[c * nb + i] = cp.acc[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Residual and analytic Jacobian. */

static cellprops *eval_all(const fr_model *m, const double *P, const double *Sw,
                           const double *X, const int8_t *flag) {
    cellprops *cp = (cellprops *)xcalloc(m->n, sizeof(cellprops));
#pragma omp parallel for schedule(static)
    for (int c = 0; c < m->n; ++c)
        eval_cell(m, c, P[c], Sw[c], X ? X[c] : 0.0, flag ? flag[c] : 0, &cp[c]);
    return cp;
}

/* add a to the (eq, unknown) entry of block (row, col) */
static void jadd(const fr_model *m, double *val, int row, int col, int eq, int u, double a) {
    if (!val) return;
    int q = blk(m, row, col);
    val[((size_t)q * m->nb + eq) * m->nb + u] += a;
}

/* Flux across the face K -> L (K < L) with transmissibility T: single-point
 * phase-potential upstream weighting, K upwind on ties, and the arithmetic
 * mean of the two cells' gravity densities (readings: the paper fixes neither).  Adds
 * +F to row K, -F to row L, and the derivatives to the four blocks. */
static void add_face(const fr_model *m, const cellprops *cp, const double *P, int K, int L,
                     double T, double *R, double *val) {
    if (T == 0.0) return;
    int nb = m->nb, np = m->np;
    double dz = m->depth[K] - m->depth[L];
    double dphi[3], ddK[3][3], ddL[3][3];
    int upK[3];
    for (int j = 0; j < np; ++j) {
        dphi[j] = (P[K] - P[L]) - 0.5 * (cp[K].gam[j] + cp[L].gam[j]) * dz;
        for (int u = 0; u < nb; ++u) {
            ddK[j][u] = (u == 0 ? 1.0 : 0.0) - 0.5 * cp[K].dgam[j][u] * dz;
            ddL[j][u] = (u == 0 ? -1.0 : 0.0) - 0.5 * cp[L].dgam[j][u] * dz;
        }
        upK[j] = dphi[j] >= 0.0;
    }
    /* component i flux = T * sum over (coefficient, phase) pairs */
    for (int i = 0; i < nb; ++i) {
        double F = 0, dFK[3] = {0, 0, 0}, dFL[3] = {0, 0, 0};
        int nterm = (i == 2) ? 2 : 1;
        for (int t = 0; t < nterm; ++t) {
            int j = (i == 2 && t == 1) ? 1 : i;       /* phase carrying the term */
            const cellprops *u = upK[j] ? &cp[K] : &cp[L];
            double coef = (i == 2 && t == 1) ? u->lamog : u->lam[j];
            const double *dcoef = (i == 2 && t == 1) ? u->dlamog : u->dlam[j];
            F += T * coef * dphi[j];
            for (int v = 0; v < nb; ++v) {
                dFK[v] += T * ((upK[j] ? dcoef[v] : 0.0) * dphi[j] + coef * ddK[j][v]);
                dFL[v] += T * ((upK[j] ? 0.0 : dcoef[v]) * dphi[j] + coef * ddL[j][v]);
            }
        }
        R[K * nb + i] += F;
        R[L * nb + i] -= F;
        for (int v = 0; v < nb; ++v) {
            jadd(m, val, K, K, i, v, dFK[v]);
            jadd(m, val, K, L, i, v, dFL[v]);
            jadd(m, val, L, K, i, v, -dFK[v]);
            jadd(m, val, L, L, i, v, -dFL[v]);
        }
    }
}

/* Perforation rates (Peaceman index, no wellbore head: a reading).  q[i] production-positive surface rate
 * of component i, dq[i][u] its derivative w.r.t. the cell unknowns and
 * dqb[i] w.r.t. the well's bottom-hole pressure.  The perforation is a
 * connection weighted by the side the flow comes from (a reading, as for
 * the faces): flow out of the cell (a producer, or an injector perforation
 * whose cell pressure exceeds the BHP) carries the cell's phases by their
 * mobilities; flow into the cell is the injected fluid with the cell's
 * total mobility. */
static void perf_rate(const fr_model *m, const cellprops *c, double Pc, int kind, double wi,
                      double pbhp, double *q, double dq[3][3], double *dqb) {
    int nb = m->nb;
    for (int i = 0; i < 3; ++i) {
        q[i] = 0; dqb[i] = 0;
        for (int u = 0; u < 3; ++u) dq[i][u] = 0;
    }
    if (kind == FR_PROD || pbhp < Pc) {
        double dp = Pc - pbhp;
        for (int i = 0; i < nb; ++i) {
            double lam = c->lam[i] + (i == 2 ? c->lamog : 0.0);
            q[i] = wi * lam * dp;
            for (int u = 0; u < nb; ++u) {
                double dl = c->dlam[i][u] + (i == 2 ? c->dlamog[u] : 0.0);
                dq[i][u] = wi * (dl * dp + lam * (u == 0 ? 1.0 : 0.0));
            }
            dqb[i] = -wi * lam;
        }
    } else {
        /* injected fluid is pure water or free gas, total cell mobility */
        int i = (kind == FR_INJ_WATER) ? 0 : 2;
        double binj = c->b[i], dbinj = c->dbP[i];
        double dp = pbhp - Pc;
        q[i] = -wi * c->lt * binj * dp;
        for (int u = 0; u < nb; ++u)
            dq[i][u] = -wi * ((c->dlt[u] * binj + c->lt * (u == 0 ? dbinj : 0.0)) * dp +
                              c->lt * binj * (u == 0 ? -1.0 : 0.0));
        dqb[i] = -wi * c->lt * binj;
    }
}

static void assemble_with(const fr_model *m, const cellprops *cp, const double *P,
                          const double *pbhp, const double *Aold, double dt, double *R,
                          double *val) {
    int n = m->n, nb = m->nb, nxy = m->nx * m->ny;
    memset(R, 0, sizeof(double) * (size_t)(n + m->nw) * nb);
    if (val) memset(val, 0, sizeof(double) * (size_t)m->nnzb * nb * nb);
    /* accumulation (Bulk::ACCU) */
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < nb; ++i) {
            R[c * nb + i] += (cp[c].acc[i] - Aold[c * nb + i]) / dt;
            for (int u = 0; u < nb; ++u) jadd(m, val, c, c, i, u, cp[c].dacc[i][u] / dt);
        }
    /* connections (BulkConn), each face once with K < L */
    for (int c = 0; c < n; ++c) {
        int i = c % m->nx, j = (c / m->nx) % m->ny, k = c / nxy;
        if (i + 1 < m->nx) add_face(m, cp, P, c, c + 1, m->tx[c], R, val);
        if (j + 1 < m->ny) add_face(m, cp, P, c, c + m->nx, m->ty[c], R, val);
        if (k + 1 < m->nz) add_face(m, cp, P, c, c + nxy, m->tz[c], R, val);
    }
    /* wells (AllWells) */
    for (int w = 0; w < m->nw; ++w) {
        int row = n + w;
        double rate_sum = 0.0, drate_b = 0.0;
        int iinj = (m->wkind[w] == FR_INJ_GAS) ? 2 : 0;
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) {
            int c = m->wpc[p];
            double q[3], dq[3][3], dqb[3];
            perf_rate(m, &cp[c], P[c], m->wkind[w], m->wi[p], pbhp[w], q, dq, dqb);
            for (int i = 0; i < nb; ++i) {
                R[c * nb + i] += q[i];
                for (int u = 0; u < nb; ++u) jadd(m, val, c, c, i, u, dq[i][u]);
                jadd(m, val, c, row, i, 0, dqb[i]);
            }
            if (m->wctrl[w] == FR_RATE) {
                rate_sum += q[iinj];
                drate_b += dqb[iinj];
                for (int u = 0; u < nb; ++u) jadd(m, val, row, c, 0, u, -dq[iinj][u]);
            }
        }
        if (m->wctrl[w] == FR_RATE) {
            R[row * nb] = -rate_sum - m->wtarget[w];
            jadd(m, val, row, row, 0, 0, -drate_b);
        } else {
            R[row * nb] = pbhp[w] - m->wtarget[w];
            jadd(m, val, row, row, 0, 0, 1.0);
        }
        for (int r = 1; r < nb; ++r) jadd(m, val, row, row, r, r, 1.0);
    }
}

void fr_assemble(const fr_model *m, const double *P, const double *Sw, const double *X,
                 const int8_t *flag, const double *pbhp, const double *Aold, double dt,
                 double *R, double *val) {
    cellprops *cp = eval_all(m, P, Sw, X, flag);
    assemble_with(m, cp, P, pbhp, Aold, dt, R, val);
    free(cp);
}

void fr_well_rates(const fr_model *m, const double *P, const double *Sw, const double *X,
                   const int8_t *flag, const double *pbhp, double *qout) {
    cellprops *cp = eval_all(m, P, Sw, X, flag);
    for (int w = 0; w < m->nw; ++w) {
        double s[3] = {0, 0, 0};
        for (int p = m->wps[w]; p < m->wps[w + 1]; ++p) {
            double q[3], dq[3][3], dqb[3];
            perf_rate(m, &cp[m->wpc[p]], P[m->wpc[p]], m->wkind[w], m->wi[p], pbhp[w], q, dq,
                      dqb);
            for (int i = 0; i < 3; ++i) s[i] += q[i];
        }
        for (int i = 0; i < 3; ++i) qout[w * 3 + i] = s[i];
    }
    free(cp);
}

/* Convergence measures (the paper defines no norm: a reading): CNV_i is the largest cell residual in
 * saturation units, MB_i the normalised global mass imbalance. */
static void conv_with(const fr_model *m, const cellprops *cp, const double *R, double dt,
                      double *cnv, double *mb) {
    int nb = m->nb;
    for (int i = 0; i < 3; ++i) { cnv[i] = 0; mb[i] = 0; }
    double sumR[3] = {0, 0, 0}, sumPV[3] = {0, 0, 0};
    for (int c = 0; c < m->n; ++c)
        for (int i = 0; i < nb; ++i) {
            double scale = cp[c].pv * cp[c].b[i];
            double v = dt * fabs(R[c * nb + i]) / scale;
            if (!(v <= cnv[i])) cnv[i] = v;   /* NaN propagates */
            sumR[i] += R[c * nb + i];
            sumPV[i] += scale;
        }
    for (int i = 0; i < nb; ++i) mb[i] = dt * fabs(sumR[i]) / sumPV[i];
}

void fr_conv(const fr_model *m, const double *P, const double *Sw, const double *X,
             const int8_t *flag, const double *R, double dt, double *cnv, double *mb) {
    cellprops *cp = eval_all(m, P, Sw, X, flag);
    conv_with(m, cp, R, dt, cnv, mb);
    free(cp);
}

/* ------------------------------------------------------------------------ */
/* Linear algebra. */

void fr_bsr_spmv(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r) {
        double acc[3] = {0, 0, 0};
        for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
            const double *a = val + (size_t)q * nb * nb;
            const double *xc = x + (size_t)colind[q] * nb;
            for (int e = 0; e < nb; ++e)
                for (int u = 0; u < nb; ++u) acc[e] += a[e * nb + u] * xc[u];
        }
        for (int e = 0; e < nb; ++e) y[(size_t)r * nb + e] = acc[e];
    }
}

/* inverse of a small nb x nb block by Gauss-Jordan with partial pivoting */
static int block_inverse(int nb, const double *a, double *inv) {
    double w[3][6];
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < 2 * nb; ++j)
            w[i][j] = (j < nb) ? a[i * nb + j] : (j - nb == i ? 1.0 : 0.0);
    for (int col = 0; col < nb; ++col) {
        int piv = col;
        for (int r = col + 1; r < nb; ++r)
            if (fabs(w[r][col]) > fabs(w[piv][col])) piv = r;
        if (w[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 2 * nb; ++j) {
                double t = w[col][j]; w[col][j] = w[piv][j]; w[piv][j] = t;
            }
        double d = w[col][col];
        for (int j = 0; j < 2 * nb; ++j) w[col][j] /= d;
        for (int r = 0; r < nb; ++r) {
            if (r == col) continue;
            double f = w[r][col];
            for (int j = 0; j < 2 * nb; ++j) w[r][j] -= f * w[col][j];
        }
    }
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) inv[i * nb + j] = w[i][nb + j];
    return 0;
}

static void block_matmul(int nb, const double *a, const double *b, double *c) {
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            double s = 0;
            for (int k = 0; k < nb; ++k) s += a[i * nb + k] * b[k * nb + j];
            c[i * nb + j] = s;
        }
}

static void block_matvec(int nb, const double *a, const double *x, double *y) {
    for (int i = 0; i < nb; ++i) {
        double s = 0;
        for (int k = 0; k < nb; ++k) s += a[i * nb + k] * x[k];
        y[i] = s;
    }
}

static int diag_pos(const int32_t *rowptr, const int32_t *colind, int r) {
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q)
        if (colind[q] == r) return q;
    return -1;
}

int fr_bj_setup(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                const double *val, double *dinv) {
    int bad = 0;
    for (int r = 0; r < nrows; ++r) {
        int q = diag_pos(rowptr, colind, r);
        if (q < 0 || block_inverse(nb, val + (size_t)q * nb * nb, dinv + (size_t)r * nb * nb))
            bad = 1;
    }
    return bad ? -1 : 0;
}

void fr_bj_apply(int32_t nrows, int32_t nb, const double *dinv, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r)
        block_matvec(nb, dinv + (size_t)r * nb * nb, x + (size_t)r * nb, y + (size_t)r * nb);
}

/* Block ILU(0) in the natural row order on the matrix's own pattern: the
 * textbook IKJ elimination restricted to existing blocks.  On exit lu holds
 * the strictly lower blocks of L (unit block diagonal implied) and the
 * upper blocks of U, with U's diagonal blocks stored inverted. */
int fr_bilu0_factor(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                    const double *val, double *lu) {
    size_t bs = (size_t)nb * nb;
    memcpy(lu, val, sizeof(double) * bs * (size_t)rowptr[nrows]);
    double tmp[9], tmp2[9];
    for (int i = 0; i < nrows; ++i) {
        for (int qk = rowptr[i]; qk < rowptr[i + 1]; ++qk) {
            int k = colind[qk];
            if (k >= i) break;
            int dk = diag_pos(rowptr, colind, k);
            /* L_ik = A_ik * inv(U_kk) */
            block_matmul(nb, lu + qk * bs, lu + dk * bs, tmp);
            memcpy(lu + qk * bs, tmp, sizeof(double) * bs);
            /* A_ij -= L_ik U_kj for j > k present in both rows */
            for (int qj = qk + 1; qj < rowptr[i + 1]; ++qj) {
                int j = colind[qj];
                for (int qkj = rowptr[k]; qkj < rowptr[k + 1]; ++qkj)
                    if (colind[qkj] == j) {
                        block_matmul(nb, lu + qk * bs, lu + qkj * bs, tmp2);
                        for (size_t e = 0; e < bs; ++e) lu[qj * bs + e] -= tmp2[e];
                    }
            }
        }
        int di = diag_pos(rowptr, colind, i);
        if (di < 0 || block_inverse(nb, lu + di * bs, tmp)) return -1;
        memcpy(lu + di * bs, tmp, sizeof(double) * bs);
    }
    return 0;
}

void fr_bilu0_solve(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                    const double *lu, const double *b, double *x) {
    size_t bs = (size_t)nb * nb;
    double t[3];
    /* forward: L y = b */
    for (int i = 0; i < nrows; ++i) {
        double s[3];
        for (int e = 0; e < nb; ++e) s[e] = b[i * nb + e];
        for (int q = rowptr[i]; q < rowptr[i + 1] && colind[q] < i; ++q) {
            block_matvec(nb, lu + q * bs, x + (size_t)colind[q] * nb, t);
            for (int e = 0; e < nb; ++e) s[e] -= t[e];
        }
        for (int e = 0; e < nb; ++e) x[i * nb + e] = s[e];
    }
    /* backward: U x = y */
    for (int i = nrows - 1; i >= 0; --i) {
        double s[3];
        int di = -1;
        for (int e = 0; e < nb; ++e) s[e] = x[i * nb + e];
        for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            if (colind[q] == i) { di = q; continue; }
            if (colind[q] < i) continue;
            block_matvec(nb, lu + q * bs, x + (size_t)colind[q] * nb, t);
            for (int e = 0; e < nb; ++e) s[e] -= t[e];
        }
        block_matvec(nb, lu + di * bs, s, t);
        for (int e = 0; e < nb; ++e) x[i * nb + e] = t[e];
    }
}

int fr_dense_solve(int32_t n, double *A, double *b) {
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[(size_t)r * n + k]) > fabs(A[(size_t)piv * n + k])) piv = r;
        if (A[(size_t)piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j];
                A[(size_t)k * n + j] = A[(size_t)piv * n + j];
                A[(size_t)piv * n + j] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        double d = A[(size_t)k * n + k];
#pragma omp parallel for schedule(static)
        for (int r = k + 1; r < n; ++r) {
            double f = A[(size_t)r * n + k] / d;
            if (f == 0.0) continue;
            A[(size_t)r * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)k * n + j];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int j = k + 1; j < n; ++j) s -= A[(size_t)k * n + j] * b[j];
        b[k] = s / A[(size_t)k * n + k];
    }
    return 0;
}

/* Dot product summed over a fixed set of chunks in a fixed order, so the
 * result does not depend on the number of threads. */
#define DOT_CHUNKS 64
static double dot(size_t n, const double *a, const double *b) {
    double part[DOT_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < DOT_CHUNKS; ++k) {
        size_t lo = n * (size_t)k / DOT_CHUNKS, hi = n * (size_t)(k + 1) / DOT_CHUNKS;
        double s = 0;
        for (size_t i = lo; i < hi; ++i) s += a[i] * b[i];
        part[k] = s;
    }
    double s = 0;
    for (int k = 0; k < DOT_CHUNKS; ++k) s += part[k];
    return s;
}

/* Right-preconditioned restarted GMRES (Saad's algorithm 6.9 / 9.5 form):
 * Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
 * matrix, x += M^-1 V y at each restart; convergence is judged on the true
 * residual ||b - A x|| / ||b||. */
int fr_gmres_bilu0(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                   const double *val, const double *b, double *x, double rtol, int32_t restart,
                   int32_t max_iter, int32_t *iters, double *relres) {
    size_t n = (size_t)nrows * nb;
    int m = restart;
    double *lu = (double *)xcalloc((size_t)rowptr[nrows] * nb * nb, sizeof(double));
    if (fr_bilu0_factor(nrows, nb, rowptr, colind, val, lu)) {
        free(lu);
        *iters = 0; *relres = NAN;
        return -1;
    }
    double *V = (double *)xcalloc(n * (m + 1), sizeof(double));
    double *H = (double *)xcalloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)xcalloc(m, sizeof(double)), *sn = (double *)xcalloc(m, sizeof(double));
    double *g = (double *)xcalloc(m + 1, sizeof(double)), *y = (double *)xcalloc(m, sizeof(double));
    double *r = (double *)xcalloc(n, sizeof(double)), *z = (double *)xcalloc(n, sizeof(double));
    double *w = (double *)xcalloc(n, sizeof(double));
    double bnorm = sqrt(dot(n, b, b));
    int total = 0, status = 1;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        *iters = 0; *relres = 0.0;
        status = 0;
        goto done;
    }
    for (;;) {
        fr_bsr_spmv(nrows, nb, rowptr, colind, val, x, r);
        for (size_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double beta = sqrt(dot(n, r, r));
        *relres = beta / bnorm;
        if (*relres <= rtol) { status = 0; break; }
        if (total >= max_iter || !isfinite(beta)) break;
        for (size_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int k = 0;
        for (; k < m && total < max_iter; ++k, ++total) {
            double *vk = V + (size_t)k * n, *vn = V + (size_t)(k + 1) * n;
            fr_bilu0_solve(nrows, nb, rowptr, colind, lu, vk, z);
            fr_bsr_spmv(nrows, nb, rowptr, colind, val, z, w);
            for (int i = 0; i <= k; ++i) {
                double *vi = V + (size_t)i * n;
                double h = dot(n, w, vi);
                H[i * m + k] = h;
                for (size_t e = 0; e < n; ++e) w[e] -= h * vi[e];
            }
            double hn = sqrt(dot(n, w, w));
            H[(k + 1) * m + k] = hn;
            if (hn > 0.0)
                for (size_t e = 0; e < n; ++e) vn[e] = w[e] / hn;
            for (int i = 0; i < k; ++i) {
                double a = H[i * m + k], c2 = H[(i + 1) * m + k];
                H[i * m + k] = cs[i] * a + sn[i] * c2;
                H[(i + 1) * m + k] = -sn[i] * a + cs[i] * c2;
            }
            double a = H[k * m + k], c2 = H[(k + 1) * m + k];
            double den = sqrt(a * a + c2 * c2);
            cs[k] = den > 0 ? a / den : 1.0;
            sn[k] = den > 0 ? c2 / den : 0.0;
            H[k * m + k] = den;
            H[(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (fabs(g[k + 1]) <= rtol * bnorm || hn == 0.0) { ++k; ++total; break; }
        }
        /* solve the triangular system and update x += M^-1 V y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * y[j];
            y[i] = s / H[i * m + i];
        }
        memset(w, 0, sizeof(double) * n);
        for (int i = 0; i < k; ++i) {
            double *vi = V + (size_t)i * n;
            for (size_t e = 0; e < n; ++e) w[e] += y[i] * vi[e];
        }
        fr_bilu0_solve(nrows, nb, rowptr, colind, lu, w, z);
        for (size_t e = 0; e < n; ++e) x[e] += z[e];
    }
    *iters = total;
done:
    free(lu); free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(z); free(w);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Newton iteration and time step (Sec. 3.2.5 and Sec. 3.3.2). */

static double tab_rs_sat(const fr_model *m, double P) {
    double v, s;
    tab_eval(m->tp, m->trs, tab_interval(m->tp, m->nrows, P), P, &v, &s);
    return v;
}

typedef struct { double *P, *Sw, *X, *pbhp; int8_t *flag; } state_t;

static void state_copy(const fr_model *m, state_t *dst, const state_t *src) {
    size_t n = (size_t)m->n;
    memcpy(dst->P, src->P, n * sizeof(double));
    memcpy(dst->Sw, src->Sw, n * sizeof(double));
    memcpy(dst->X, src->X, n * sizeof(double));
    memcpy(dst->flag, src->flag, n);
    if (m->nw) memcpy(dst->pbhp, src->pbhp, (size_t)m->nw * sizeof(double));
}

static state_t state_alloc(const fr_model *m) {
    state_t s;
    s.P = (double *)xcalloc(m->n, sizeof(double));
    s.Sw = (double *)xcalloc(m->n, sizeof(double));
    s.X = (double *)xcalloc(m->n, sizeof(double));
    s.flag = (int8_t *)xcalloc(m->n, 1);
    s.pbhp = (double *)xcalloc(m->nw, sizeof(double));
    return s;
}

static void state_free(state_t *s) { free(s->P); free(s->Sw); free(s->X); free(s->flag); free(s->pbhp); }

/* Newton update with per-cell saturation chopping, pressure clipping and
 * three-phase variable switching (readings: the paper states neither the chop nor the switch).  Returns the largest
 * applied pressure and saturation changes. */
static void newton_update(const fr_model *m, state_t *s, const double *dx, const fr_options *o,
                          double *maxdp, double *maxds) {
    int nb = m->nb;
    double mdp = 0, mds = 0;
    for (int c = 0; c < m->n; ++c) {
        double dP = dx[c * nb];
        if (dP > o->dp_max) dP = o->dp_max;
        if (dP < -o->dp_max) dP = -o->dp_max;
        double dSw = dx[c * nb + 1];
        double dX = (nb == 3) ? dx[c * nb + 2] : 0.0;
        int sat = (nb == 3 && s->flag[c] == FR_SAT);
        double smax = fabs(dSw);
        if (sat && fabs(dX) > smax) smax = fabs(dX);
        if (smax > o->ds_max) {
            double f = o->ds_max / smax;
            dSw *= f;
            if (sat) dX *= f;
        }
        s->P[c] += dP;
        s->Sw[c] += dSw;
        s->X[c] += dX;
        if (fabs(dP) > mdp) mdp = fabs(dP);
        if (fabs(dSw) > mds) mds = fabs(dSw);
        if (sat && fabs(dX) > mds) mds = fabs(dX);
        if (!isfinite(dP) || !isfinite(dSw) || !isfinite(dX)) mdp = NAN;
        if (nb == 3) {
            if (sat && s->X[c] < 0.0) {
                s->flag[c] = FR_UNSAT;
                s->X[c] = tab_rs_sat(m, s->P[c]);
            } else if (!sat && s->X[c] > tab_rs_sat(m, s->P[c])) {
                s->flag[c] = FR_SAT;
                s->X[c] = 0.0;
            }
        }
    }
    for (int w = 0; w < m->nw; ++w) {
        double d = dx[(size_t)(m->n + w) * nb];
        if (d > o->dp_max) d = o->dp_max;
        if (d < -o->dp_max) d = -o->dp_max;
        s->pbhp[w] += d;
        if (fabs(d) > mdp) mdp = fabs(d);
        if (!isfinite(d)) mdp = NAN;
    }
    *maxdp = mdp;
    *maxds = mds;
}

/* Well equations are measured in pressure units: the residual of the well
 * row divided by its derivative with respect to the bottom-hole pressure
 * (1 for a BHP row, the summed perforation productivity for a rate row). */
static int well_rows_ok(const fr_model *m, const double *R, const double *val, double tol) {
    int nb = m->nb;
    for (int w = 0; w < m->nw; ++w) {
        int row = m->n + w;
        double d = fabs(val[(size_t)blk(m, row, row) * nb * nb]);
        double r = fabs(R[(size_t)row * nb]) / (d > 0.0 ? d : 1.0);
        if (!(r <= tol)) return 0;
    }
    return 1;
}

static int solve_linear(const fr_model *m, const double *val, const double *R, double *dx,
                        const fr_options *o, int *iters) {
    int nrows = m->n + m->nw, nb = m->nb;
    size_t nu = (size_t)nrows * nb;
    double *rhs = (double *)xcalloc(nu, sizeof(double));
    for (size_t i = 0; i < nu; ++i) rhs[i] = -R[i];
    int ok = 0;
    if (o->linsolve) {
        int32_t it = 0;
        ok = o->linsolve(o->linsolve_ctx, nrows, nb, m->rowptr, m->colind, val, rhs, dx, &it) == 0;
        *iters = it;
    } else if ((int)nu <= o->dense_max) {
        double *A = (double *)xcalloc(nu * nu, sizeof(double));
        for (int r = 0; r < nrows; ++r)
            for (int q = m->rowptr[r]; q < m->rowptr[r + 1]; ++q)
                for (int e = 0; e < nb; ++e)
                    for (int u = 0; u < nb; ++u)
                        A[((size_t)r * nb + e) * nu + (size_t)m->colind[q] * nb + u] =
                            val[((size_t)q * nb + e) * nb + u];
        ok = fr_dense_solve((int)nu, A, rhs) == 0;
        memcpy(dx, rhs, nu * sizeof(double));
        *iters = 1;
        free(A);
    } else {
        double relres;
        memset(dx, 0, nu * sizeof(double));
        int st = fr_gmres_bilu0(nrows, nb, m->rowptr, m->colind, val, rhs, dx, o->lin_rtol,
                                o->restart, o->max_lin, iters, &relres);
        ok = (st == 0) || (isfinite(relres) && relres < 1.0);
    }
    for (size_t i = 0; i < nu && ok; ++i)
        if (!isfinite(dx[i])) ok = 0;
    free(rhs);
    return ok;
}

/* 1 when every saturation (Sw, So, Sg) of the state lies in [-1e-6, 1 + 1e-6] */
static int physical(const fr_model *m, const state_t *s) {
    for (int c = 0; c < m->n; ++c) {
        double sw = s->Sw[c];
        double sg = (m->nb == 3 && s->flag[c] == FR_SAT) ? s->X[c] : 0.0;
        double so = 1.0 - sw - sg;
        double lo = fmin(fmin(sw, so), sg), hi = fmax(fmax(sw, so), sg);
        if (!(lo >= -1e-6 && hi <= 1.0 + 1e-6)) return 0;
    }
    return 1;
}

/* Newton iterations for one sub-step; 1 on convergence. */
static int newton(const fr_model *m, state_t *s, double dt, const fr_options *o, fr_report *rep) {
    int n = m->n, nb = m->nb;
    size_t nu = (size_t)(n + m->nw) * nb;
    double *Aold = (double *)xcalloc((size_t)n * nb, sizeof(double));
    double *R = (double *)xcalloc(nu, sizeof(double));
    double *val = (double *)xcalloc((size_t)m->nnzb * nb * nb, sizeof(double));
    double *dx = (double *)xcalloc(nu, sizeof(double));
    fr_accum(m, s->P, s->Sw, s->X, s->flag, Aold);
    double last_dp = INFINITY, last_ds = INFINITY;
    int ok = 0;
    for (int it = 0;; ++it) {
        double t0 = omp_get_wtime();
        cellprops *cp = eval_all(m, s->P, s->Sw, s->X, s->flag);
        assemble_with(m, cp, s->P, s->pbhp, Aold, dt, R, val);
        conv_with(m, cp, R, dt, rep->cnv, rep->mb);
        free(cp);
        double t1 = omp_get_wtime();
        rep->t_assemble += t1 - t0;
        int finite = 1;
        for (size_t i = 0; i < nu; ++i)
            if (!isfinite(R[i])) { finite = 0; break; }
        if (!finite) break;
        int conv = it > 0 && last_dp <= o->tol_dp && last_ds <= o->tol_ds &&
                   well_rows_ok(m, R, val, o->tol_well);
        for (int i = 0; i < nb; ++i)
            conv = conv && rep->cnv[i] <= o->tol_cnv && rep->mb[i] <= o->tol_mb;
        /* a root whose saturations leave [0, 1] by more than 1e-6 is not a
         * physical state: the sub-step fails (a reading; the paper counts
         * non-physical results among the failures that cut the step) */
        if (conv) { ok = physical(m, s); break; }
        if (it >= o->max_newton) break;
        int li = 0;
        int lin_ok = solve_linear(m, val, R, dx, o, &li);
        double t2 = omp_get_wtime();
        rep->t_linear += t2 - t1;
        rep->linear_iters += li;
        rep->newton_iters += 1;
        if (!lin_ok) break;
        newton_update(m, s, dx, o, &last_dp, &last_ds);
        rep->t_update += omp_get_wtime() - t2;
        if (!isfinite(last_dp)) break;
    }
    free(Aold); free(R); free(val); free(dx);
    return ok;
}

int fr_step(const fr_model *m, double *P, double *Sw, double *X, int8_t *flag, double *pbhp,
            double dt, const fr_options *opt, fr_report *rep) {
    memset(rep, 0, sizeof *rep);
    state_t cur = {P, Sw, X, pbhp, flag};
    state_t start = state_alloc(m), sub = state_alloc(m);
    state_copy(m, &start, &cur);
    double remaining = dt, h = dt;
    int status = 0;
    while (remaining > 1e-12 * dt) {
        double try_dt = h < remaining ? h : remaining;
        state_copy(m, &sub, &cur);
        if (newton(m, &cur, try_dt, opt, rep)) {
            remaining -= try_dt;
            if (rep->nsub < FR_MAX_SUB) rep->dt_sub[rep->nsub] = try_dt;
            rep->nsub++;
        } else {
            state_copy(m, &cur, &sub);
            rep->cuts++;
            if (rep->cuts > opt->max_cuts) {
                state_copy(m, &cur, &start);
                status = 1;
                break;
            }
            h = 0.5 * try_dt;
        }
    }
    rep->converged = (status == 0);
    state_free(&start);
    state_free(&sub);
    return status;
}
