// fim_api.cpp - host runtime behind the C ABI (include/fim.h): context and
// device memory, static pattern, the Newton driver (paper Sec. 3.2.5), the
// time-step driver with conditional returns (Sec. 3.3.2) and the GMRES
// driver (Sec. 5.1, Sec. 3.3.3).  The host only orders launches, reads a
// few scalars per iteration and solves the small Hessenberg least-squares
// problem of GMRES; every vector and matrix operation is a HIP kernel.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <stdexcept>
#include <system_error>
#include <thread>
#include <type_traits>
#include <vector>

#include "fim.h"
#include "fim_internal.h"

using namespace fim;

namespace {

thread_local std::string g_err;

struct ArgError {};
struct HipError {};
struct StateError {};

void set_err(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

#define HIPCHECK(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_err("HIP error '%s' in %s (%s:%d)", hipGetErrorString(e_), #call, __FILE__, \
                    __LINE__);                                                            \
            throw HipError();                                                             \
        }                                                                                 \
    } while (0)

#define REQUIRE(cond, ...)        \
    do {                          \
        if (!(cond)) {            \
            set_err(__VA_ARGS__); \
            throw ArgError();     \
        }                         \
    } while (0)

template <typename F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const ArgError &) {
        return FIM_E_ARG;
    } catch (const StateError &) {
        return FIM_E_STATE;
    } catch (const HipError &) {
        return FIM_E_HIP;
    } catch (const std::bad_alloc &) {
        set_err("host out of memory");
        return FIM_E_NOMEM;
    } catch (...) {
        set_err("unexpected internal error");
        return FIM_E_HIP;
    }
}

// scalar slots in the device/pinned scalar area
enum { S_CONV = 0, S_UPD = 16, S_NORM = 20, S_RES = 24, S_COUNT = 32 };

// how far a saturation of a converged iterate may lie outside [0, 1]
constexpr double kSatSlack = 1e-6;

}  // namespace

struct fim_ctx {
    hipStream_t s = nullptr;          // the context's own stream
    hipStream_t s2 = nullptr;         // the ILU(0) factorisation beside the AMG setup
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipStream_t user_s = nullptr;     // the caller's stream the work is ordered after
    hipEvent_t ev_user = nullptr;
    hipGraphExec_t step_exec[kMaxRestart] = {};   // Arnoldi step j after its SpMV
    hipGraphExec_t step_full[kMaxRestart] = {};   // Arnoldi step j with its SpMV
    int dev = 0;
    fim_options opt{};
    Grid g{};
    int n = 0, nb = 0, nw = 0, nperf = 0, nrows = 0, nnzb = 0, m = 0;
    long nvec = 0;
    Phys phys{};
    std::vector<int> wkind, wctrl, wps, perf_src;   // perf_src: sorted -> input index
    std::vector<double> wtarget;
    std::vector<void *> owned;
    // device
    double *dx = nullptr, *dy = nullptr, *dz = nullptr, *kx = nullptr, *ky = nullptr,
           *kz = nullptr, *poro = nullptr, *tab = nullptr;
    double *vol = nullptr, *depth = nullptr, *pvref = nullptr, *tx = nullptr, *ty = nullptr,
           *tz = nullptr;
    int *dwkind = nullptr, *dwctrl = nullptr, *dwps = nullptr, *pcell = nullptr,
        *pwell = nullptr, *cps = nullptr, *cperf = nullptr;
    double *dwtarget = nullptr, *wi = nullptr, *wrw = nullptr, *wskin = nullptr;
    double *P = nullptr, *Sw = nullptr, *X = nullptr, *pbhp = nullptr;
    int8_t *flag = nullptr;
    double *sP[2] = {}, *sSw[2] = {}, *sX[2] = {}, *spb[2] = {};
    int8_t *sflag[2] = {};
    double *rec = nullptr, *aold = nullptr, *wmeas = nullptr;
    int *rowptr = nullptr, *colind = nullptr, *diagpos = nullptr;
    double *val = nullptr, *R = nullptr, *dinv = nullptr;
    int *bad = nullptr;
    double *V = nullptr, *Z = nullptr, *w = nullptr, *z = nullptr, *x = nullptr, *r = nullptr,
           *t = nullptr, *b = nullptr, *H = nullptr, *tmp = nullptr, *ydev = nullptr;
    // pressure AMG of the CPR preconditioner
    std::vector<AmgLevel> lv;
    std::vector<const int *> cfs_ptr, cfs_idx;     // coarse slot -> fine slots, per level
    double *Mden = nullptr, *Minv = nullptr, *colk = nullptr, *wq = nullptr;
    double *ap = nullptr;                           // [nnzb][nb] pressure column of A
    // weights of the first CPR stage: restriction (null: the quasi-IMPES
    // weights wq) and prolongation (null: the pressure slot)
    const double *cpr_rw = nullptr, *cpr_pw = nullptr;
    double *e0w = nullptr;                          // [n][nb] (1, 0, ..): the pressure component
    // block-Jacobi ILU(0): tiles, factors and the CPR second-stage scratch
    IluTiles ilu{};
    int ilu_dims[3] = {0, 0, 0};
    std::vector<int> perf_cell_h;                   // perforated cell of each perforation
    double *lu = nullptr;
    size_t lu_elems = 0, lu32_elems = 0;            // allocated elements of lu, lu32
    // mixed precision: single-precision copies for the inner solves
    bool mixed = false;
    int m32 = 0;
    float *val32 = nullptr, *V32 = nullptr, *Z32 = nullptr, *w32 = nullptr, *lu32 = nullptr,
          *ap32 = nullptr;
    int *ilu_bad = nullptr;
    int sub_root = -1;                              // first level of the fused sub-cycle
    int *sub_ops = nullptr;                         // [kSubOps] its phase list
    AmgSub sub{};
    int *amg_bad = nullptr;
    bool exact_on = false;        // the coarsest level is solved by slabs (AmgExact)
    AmgExact ex{};
    int *split0 = nullptr;                          // natural cell -> level-0 split index
    int *colsplit = nullptr;                        // [nnzb] column -> level-0 entry
    int *reorth = nullptr;
    double *partials = nullptr, *scal = nullptr;
    double *pin = nullptr;        // pinned host: scalars, H columns, y
    size_t pin_len = 0;
    bool state_set = false, jac_ready = false, prec_ready = false;
    hipEvent_t ev[4] = {};
    hipEvent_t colev[kMaxRestart] = {};
    std::vector<hipEvent_t> spmv_ev;
    int spmv_used = 0;
    double spmv_ms = 0.0;
    int spmv_calls = 0;
    double gs_vectors = 0.0;                  // basis vectors orthogonalised against (step)
    long spmv_seq = 0;                        // solver SpMVs since the context was made
    // discrete adjoint: the state after every accepted sub-step of the
    // forward run and the work arrays of the backward sweep
    double *wi_dk = nullptr;                        // [nperf] 1: WI ~ k (Peaceman), 0: explicit
    int *tperm = nullptr;                           // [nnzb] block of J^T -> block of J
    double *valT = nullptr;                         // [nnzb][nb][nb]
    double *lam[2] = {}, *arhs = nullptr, *grad = nullptr, *objp = nullptr, *objw = nullptr,
           *qobs = nullptr;
    size_t qobs_len = 0;
    struct Ckpt {
        double *P, *Sw, *X, *pbhp;
        int8_t *flag;
    };
    std::vector<Ckpt> ckpt;                         // sub-step states of the backward sweep
    std::vector<Ckpt> seg;                          // segment-start states (checkpointing)
    std::vector<double> wi_explicit;                // per sorted perforation: explicit WI or 0
    double top = 0.0;

    Wells wells() const {
        Wells W;
        W.nw = nw;
        W.kind = dwkind;
        W.ctrl = dwctrl;
        W.target = dwtarget;
        W.wps = dwps;
        W.pcell = pcell;
        W.pwell = pwell;
        W.wi = wi;
        W.cps = cps;
        W.cperf = cperf;
        return W;
    }
    Sys sys() const { return Sys{rowptr, colind, diagpos, val, R}; }

    template <typename T>
    T *alloc(size_t count) {
        void *p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            set_err("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
            throw std::bad_alloc();
        }
        owned.push_back(p);
        return static_cast<T *>(p);
    }
    template <typename T>
    T *upload(const T *src, size_t count) {
        T *d = alloc<T>(count);
        if (src && count) HIPCHECK(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, s));
        return d;
    }
    void sync() { HIPCHECK(hipStreamSynchronize(s)); }
    void release(void *p) {
        if (!p) return;
        auto it = std::find(owned.begin(), owned.end(), p);
        if (it != owned.end()) owned.erase(it);
        (void)hipFree(p);
    }

    void drop_graphs() {
        for (auto *set : {step_exec, step_full})
            for (int j = 0; j < kMaxRestart; ++j)
                if (set[j]) {
                    (void)hipGraphExecDestroy(set[j]);
                    set[j] = nullptr;
                }
    }

    ~fim_ctx() {
        if (s) (void)hipStreamSynchronize(s);
        drop_graphs();
        for (void *p : owned) (void)hipFree(p);
        if (pin) (void)hipHostFree(pin);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : colev)
            if (e) (void)hipEventDestroy(e);
        for (auto &e : spmv_ev) (void)hipEventDestroy(e);
        if (ev_user) (void)hipEventDestroy(ev_user);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (s2) (void)hipStreamDestroy(s2);
        if (s) (void)hipStreamDestroy(s);
    }
};

// ---------------------------------------------------------------------------
// validation and setup

static void check_options(const fim_options *o) {
    REQUIRE(o, "options pointer is NULL");
    REQUIRE(o->restart >= 1 && o->restart <= kMaxRestart, "restart must be in [1, %d]",
            kMaxRestart);
    REQUIRE(o->max_lin >= 1 && o->max_newton >= 1 && o->max_cuts >= 0,
            "max_lin, max_newton >= 1 and max_cuts >= 0 required");
    REQUIRE(o->ds_max > 0 && o->dp_max > 0 && o->lin_rtol > 0 && o->lin_rtol < 1,
            "ds_max, dp_max > 0 and 0 < lin_rtol < 1 required");
    REQUIRE(o->precond >= FIM_PREC_BJ && o->precond <= FIM_PREC_CPR_ILU0,
            "unknown preconditioner %d", o->precond);
    REQUIRE(o->tile_nx >= 0 && o->tile_ny >= 0 && o->tile_nz >= 0, "tile sizes must be >= 0");
    REQUIRE((o->amg_cycle >= 0 && o->amg_cycle <= 2) || o->amg_cycle >= 16 || o->amg_cycle <= -16,
            "amg_cycle must be 0, 1, 2 or a level size >= 16 or <= -16");
    REQUIRE(o->amg_sweeps >= 0 && o->amg_sweeps <= 8, "amg_sweeps must be in [0, 8]");
    REQUIRE(o->graphs == 0 || o->graphs == 1, "graphs must be 0 or 1");
    REQUIRE(o->forcing == 0 || o->forcing == 1, "forcing must be 0 or 1");
    REQUIRE(o->precision == FIM_FP64 || o->precision == FIM_MIXED, "unknown precision mode %d",
            o->precision);
    REQUIRE(o->precision == FIM_FP64 || o->precond == FIM_PREC_ILU0 ||
                o->precond == FIM_PREC_CPR_ILU0,
            "mixed precision needs an ILU(0) preconditioner (FIM_PREC_ILU0 or FIM_PREC_CPR_ILU0)");
    REQUIRE(o->amg_fused <= (1 << 20), "amg_fused must be at most 2^20 cells");
    REQUIRE(o->gs_refine >= -1 && o->gs_refine <= 1, "gs_refine must be -1, 0 or 1");
    REQUIRE(o->profile >= 0, "profile must be >= 0");
    REQUIRE(o->amg_exact >= -1 && o->amg_exact <= (1 << 20), "amg_exact must be in [-1, 2^20]");
    REQUIRE(o->amg_exact_mode == 0 || o->amg_exact_mode == 1, "amg_exact_mode must be 0 or 1");
}

static void build_pattern(fim_ctx *c, std::vector<int> &rp, std::vector<int> &ci,
                          std::vector<int> &dp, const std::vector<std::vector<int>> &cell_wells,
                          const std::vector<int> &sorted_cells) {
    const int n = c->n, nx = c->g.nx, ny = c->g.ny, nz = c->g.nz, nxy = nx * ny;
    rp.assign(c->nrows + 1, 0);
    ci.clear();
    dp.assign(c->nrows, -1);
    for (int cell = 0; cell < n; ++cell) {
        const int i = cell % nx, j = (cell / nx) % ny, k = cell / nxy;
        // ascending columns: -z, -y, -x, diagonal, +x, +y, +z, well columns
        if (k > 0) ci.push_back(cell - nxy);
        if (j > 0) ci.push_back(cell - nx);
        if (i > 0) ci.push_back(cell - 1);
        dp[cell] = (int)ci.size();
        ci.push_back(cell);
        if (i + 1 < nx) ci.push_back(cell + 1);
        if (j + 1 < ny) ci.push_back(cell + nx);
        if (k + 1 < nz) ci.push_back(cell + nxy);
        for (int wl : cell_wells[cell]) ci.push_back(n + wl);
        rp[cell + 1] = (int)ci.size();
    }
    for (int wl = 0; wl < c->nw; ++wl) {
        for (int p = c->wps[wl]; p < c->wps[wl + 1]; ++p) ci.push_back(sorted_cells[p]);
        dp[n + wl] = (int)ci.size();
        ci.push_back(n + wl);
        rp[n + wl + 1] = (int)ci.size();
    }
}

static void alloc_krylov(fim_ctx *c, int m) {
    c->release(c->V);
    c->release(c->Z);
    c->release(c->H);
    c->V = c->Z = c->H = nullptr;
    c->m = m;
    c->V = c->alloc<double>((size_t)(m + 1) * c->nvec);
    c->Z = c->alloc<double>((size_t)(m + 1) * c->nvec);
    c->H = c->alloc<double>((size_t)(m + 1) * (kMaxRestart + 2));
}

// Whether the level just built (nx x ny x nz cells; well slots at natural
// cells slot_cell, of wells slot_well, ranges sps) can be the coarsest,
// solved exactly by slabs: at most amg_exact cells (option; <= 0 = never,
// the default), slabs along the longest axis of at most
// kSlabMax cells and wells, and every well's cells in one slab.  On
// success fills c->ex (device arrays uploaded) and sets c->exact_on.
static bool plan_exact(fim_ctx *c, int nx, int ny, int nz, const std::vector<int> &slot_cell,
                       const std::vector<int> &slot_well, const std::vector<int> &sps) {
    if (c->opt.amg_exact <= 0) return false;           // 0: the default, off
    const long cells = (long)nx * ny * nz;
    if (cells > c->opt.amg_exact) return false;
    const int dims[3] = {nx, ny, nz};
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (dims[a] > dims[axis]) axis = a;
    AmgExact E{};
    E.axis = axis;
    E.nslab = dims[axis];
    E.nu = axis == 0 ? ny : nx;
    E.nv = axis == 2 ? ny : nz;
    E.ncs = E.nu * E.nv;
    const int nw = c->nw;
    std::vector<int> wslab(nw, -1);
    for (int w = 0; w < nw; ++w)
        for (int q = sps[w]; q < sps[w + 1]; ++q) {
            const int cn = slot_cell[q];
            const int ci[3] = {cn % nx, (cn / nx) % ny, cn / (nx * ny)};
            if (wslab[w] >= 0 && wslab[w] != ci[axis]) return false;   // a well across slabs
            wslab[w] = ci[axis];
        }
    std::vector<int> swp(E.nslab + 1, 0), sw, wrank(std::max(nw, 1), 0);
    for (int w = 0; w < nw; ++w)
        if (wslab[w] >= 0) swp[wslab[w] + 1]++;
    for (int b = 0; b < E.nslab; ++b) swp[b + 1] += swp[b];
    int mwell = 0;
    for (int b = 0; b < E.nslab; ++b) mwell = std::max(mwell, swp[b + 1] - swp[b]);
    E.mmax = E.ncs + mwell;
    if (E.mmax > kSlabMax || (long)E.nslab * E.mmax > kExactSlabDoubles) return false;
    if ((int)swp[E.nslab] != nw) return false;             // a well without a slot
    sw.resize(std::max(nw, 1));
    {
        std::vector<int> fill(swp.begin(), swp.end() - 1);
        for (int w = 0; w < nw; ++w) {
            wrank[w] = fill[wslab[w]] - swp[wslab[w]];
            sw[fill[wslab[w]]++] = w;
        }
    }
    E.swp = c->upload(swp.data(), swp.size());
    E.sw = c->upload(sw.data(), sw.size());
    E.wrank = c->upload(wrank.data(), wrank.size());
    c->sync();
    c->ex = E;
    c->exact_on = true;
    return true;
}

// Structured aggregation hierarchy of the pressure AMG (built once): level
// dimensions halve (rounding up) until a level has at most kCoarseMax cells;
// each well keeps one slot per distinct perforated cell of every level.
static void build_amg(fim_ctx *c, const std::vector<int> &sorted_cells,
                      const std::vector<int> &pwell_h) {
    int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    const int nw = c->nw;
    std::vector<int> slot_cell = sorted_cells, slot_well = pwell_h, sps = c->wps;
    c->cfs_ptr.push_back(nullptr);
    c->cfs_idx.push_back(nullptr);
    for (;;) {
        AmgLevel L{};
        L.nx = nx;
        L.ny = ny;
        L.nz = nz;
        L.nxp = nx + (nx & 1);
        L.half = L.nxp * ny * nz / 2;
        L.nw = nw;
        L.nslot = (int)slot_cell.size();
        auto magic = [](long d) { return (unsigned long long)(((1ULL << 40) + d - 1) / d); };
        L.mnx = magic(nx);
        L.mny = magic(ny);
        L.mnxp = magic(L.nxp);
        // the multiply-shift divisions of the cycle kernels are exact while
        // numerator * divisor < 2^40
        REQUIRE((double)L.nxp * ny * nz * L.nxp < 1099511627776.0 &&
                    (double)ny * nz * ny < 1099511627776.0 &&
                    (double)nx * ny * nz * nx < 1099511627776.0,
                "grid %d x %d x %d too large for the AMG index arithmetic", nx, ny, nz);
        const int ncs = 2 * L.half;
        auto split = [&](int cn) {
            const int i = cn % nx, j = (cn / nx) % ny, k = cn / (nx * ny);
            const int cc = i + L.nxp * (j + ny * k);
            return (((i + j + k) & 1) ? L.half : 0) + (cc >> 1);
        };
        std::vector<int> scell(L.nslot), cps(ncs + 1, 0), cslot(L.nslot);
        for (int q = 0; q < L.nslot; ++q) {
            scell[q] = split(slot_cell[q]);
            cps[scell[q] + 1]++;
        }
        for (int q = 0; q < ncs; ++q) cps[q + 1] += cps[q];
        {
            std::vector<int> fill(cps.begin(), cps.end() - 1);
            for (int q = 0; q < L.nslot; ++q) cslot[fill[scell[q]]++] = q;
        }
        L.a = c->alloc<double>((size_t)7 * ncs);
        launch_scale_copy(c->s, ncs, nullptr, 1.0, L.a);
        launch_scale_copy(c->s, 6L * ncs, nullptr, 0.0, L.a + ncs);
        L.aww = c->alloc<double>(std::max(nw, 1));
        L.acw = c->alloc<double>(std::max(L.nslot, 1));
        L.awc = c->alloc<double>(std::max(L.nslot, 1));
        L.x = c->alloc<double>(ncs + nw);
        L.b = c->alloc<double>(ncs + nw);
        L.xs = c->alloc<double>(std::max(nw, 1));
        launch_scale_copy(c->s, ncs + nw, nullptr, 0.0, L.x);
        launch_scale_copy(c->s, ncs + nw, nullptr, 0.0, L.b);
        if (c->lv.empty()) {
            std::vector<int> sp(c->n);
            for (int cn = 0; cn < c->n; ++cn) sp[cn] = split(cn);
            c->split0 = c->upload(sp.data(), sp.size());
        }
        L.sps = c->upload(sps.data(), sps.size());
        L.scell = c->upload(scell.data(), scell.size());
        L.swell = c->upload(slot_well.data(), slot_well.size());
        L.cps = c->upload(cps.data(), cps.size());
        L.cslot = c->upload(cslot.data(), cslot.size());
        c->sync();                  // the host vectors above are temporaries
        c->lv.push_back(L);
        if (c->lv.size() > 1 && plan_exact(c, nx, ny, nz, slot_cell, slot_well, sps)) break;
        if ((long)nx * ny * nz <= kCoarseMax || (nx == 1 && ny == 1 && nz == 1)) break;
        // next level: coarse dimensions and the well slots they keep
        const int cnx = (nx + 1) / 2, cny = (ny + 1) / 2, cnz = (nz + 1) / 2;
        std::vector<int> ncell, nwell, nsps(nw + 1, 0), fine_to_coarse(L.nslot);
        for (int w = 0; w < nw; ++w) {
            std::vector<int> cc;
            for (int q = sps[w]; q < sps[w + 1]; ++q) {
                const int cn = slot_cell[q];
                const int i = cn % nx, j = (cn / nx) % ny, k = cn / (nx * ny);
                cc.push_back(i / 2 + cnx * (j / 2 + cny * (k / 2)));
            }
            std::vector<int> uniq = cc;
            std::sort(uniq.begin(), uniq.end());
            uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
            const int base = (int)ncell.size();
            for (int u : uniq) {
                ncell.push_back(u);
                nwell.push_back(w);
            }
            for (int q = sps[w]; q < sps[w + 1]; ++q)
                fine_to_coarse[q] = base + (int)(std::lower_bound(uniq.begin(), uniq.end(),
                                                                  cc[q - sps[w]]) - uniq.begin());
            nsps[w + 1] = (int)ncell.size();
        }
        std::vector<int> fptr(ncell.size() + 1, 0), fidx(L.nslot);
        for (int q = 0; q < L.nslot; ++q) fptr[fine_to_coarse[q] + 1]++;
        for (size_t q = 0; q < ncell.size(); ++q) fptr[q + 1] += fptr[q];
        {
            std::vector<int> fill(fptr.begin(), fptr.end() - 1);
            for (int q = 0; q < L.nslot; ++q) fidx[fill[fine_to_coarse[q]]++] = q;
        }
        c->cfs_ptr.push_back(c->upload(fptr.data(), fptr.size()));
        c->cfs_idx.push_back(c->upload(fidx.data(), std::max<size_t>(fidx.size(), 1)));
        c->sync();
        nx = cnx;
        ny = cny;
        nz = cnz;
        slot_cell.swap(ncell);
        slot_well.swap(nwell);
        sps.swap(nsps);
    }
    c->amg_bad = c->alloc<int>(1);
    if (c->exact_on) {
        c->ex.bad = c->amg_bad;
        // (the padding is read past the last row by the inverse's chunked loads)
        const size_t nbinv = (size_t)c->ex.nslab * c->ex.mmax * c->ex.mmax;
        c->ex.binv = c->alloc<double>(nbinv + kSlabMax);
        HIPCHECK(hipMemsetAsync(c->ex.binv, 0, (nbinv + kSlabMax) * sizeof(double), c->s));
        HIPCHECK(exact_allow_lds());            // the same value for every context
        // mode 0: room for the level's dense inverse (rows and columns in
        // storage order; padded ones stay zero)
        const AmgLevel &Lc = c->lv.back();
        AmgExact &E = c->ex;
        E.nst = 2 * Lc.half + Lc.nw;
        E.ncol = E.nslab * E.ncs + Lc.nw;
        E.ldx = (E.ncol + 1) & ~1;
        E.twist = E.nslab / 2;
        E.X = nullptr;
        E.cmap = nullptr;
        if (c->opt.amg_exact_mode == 0 && E.ldx <= kExactGemvCols) {
            // column f of slab b, position p (cells by their in-slab position,
            // then the slab's wells) -> the level's storage index
            std::vector<int> swp(E.nslab + 1), sw(std::max(Lc.nw, 1)), cmap(E.ncol);
            HIPCHECK(hipMemcpy(swp.data(), E.swp, swp.size() * sizeof(int), hipMemcpyDeviceToHost));
            HIPCHECK(hipMemcpy(sw.data(), E.sw, sw.size() * sizeof(int), hipMemcpyDeviceToHost));
            for (int b = 0; b < E.nslab; ++b) {
                const int m = E.ncs + swp[b + 1] - swp[b];
                for (int p = 0; p < m; ++p) {
                    int st;
                    if (p >= E.ncs) {
                        st = 2 * Lc.half + sw[swp[b] + p - E.ncs];
                    } else {
                        const int u = p % E.nu, v = p / E.nu;
                        const int i = E.axis == 0 ? b : u, j = E.axis == 0 ? u : (E.axis == 1 ? b : v),
                                  k = E.axis == 2 ? b : v;
                        st = (((i + j + k) & 1) ? Lc.half : 0) + ((i + Lc.nxp * (j + Lc.ny * k)) >> 1);
                    }
                    cmap[(size_t)b * E.ncs + swp[b] + p] = st;
                }
            }
            E.cmap = c->upload(cmap.data(), cmap.size());
            E.X = c->alloc<double>((size_t)E.nst * E.ldx);
            HIPCHECK(hipMemsetAsync(E.X, 0, (size_t)E.nst * E.ldx * sizeof(double), c->s));
        }
    } else {
        const AmgLevel &Lc = c->lv.back();
        const size_t n = 2 * (size_t)Lc.half + Lc.nw;
        c->Mden = c->alloc<double>(n * n);
        c->Minv = c->alloc<double>(n * n);
        c->colk = c->alloc<double>(n);
    }
    HIPCHECK(dense_allow_lds());                // the same value for every context
    c->wq = c->alloc<double>((size_t)c->n * c->nb);
    c->ap = c->alloc<double>((size_t)c->nnzb * c->nb);
}

// The coarsest level's solver from its current operator: the slab
// factorisation, or the dense inverse.
static void coarsest_setup(fim_ctx *c) {
    if (c->exact_on) {
        launch_amg_exact_factor(c->s, c->lv.back(), c->ex);
        if (c->ex.X) launch_amg_exact_inverse(c->s, c->lv.back(), c->ex);
    } else launch_amg_coarsest_setup(c->s, c->lv.back(), c->Mden, c->Minv, c->colk, c->amg_bad);
}

// x = A^-1 b on the slab-solved coarsest level: by its dense inverse over
// the whole device, or by substitution over the slabs in one workgroup.
static void exact_apply(fim_ctx *c, const AmgLevel &L) {
    if (c->ex.X) launch_amg_exact_gemv(c->s, L, c->ex);
    else launch_amg_exact_solve(c->s, L, c->ex);
}

static void build_subcycle(fim_ctx *c);
static void build_ilu(fim_ctx *c);
static void ensure_mixed(fim_ctx *c);

static int create_impl(const fim_grid *grid, const fim_rock *rock, const fim_fluid *fl,
                       int32_t nwells, const fim_well *wells, const fim_options *opt,
                       void *stream, fim_ctx **out) {
    REQUIRE(out, "out pointer is NULL");
    *out = nullptr;
    REQUIRE(grid && rock && fl, "grid, rock and fluid are required");
    REQUIRE(grid->nx >= 1 && grid->ny >= 1 && grid->nz >= 1, "grid dimensions must be >= 1");
    const long nl = (long)grid->nx * grid->ny * grid->nz;
    REQUIRE(nl < (1L << 28), "grid too large (%ld cells, at most 2^28 - 1)", nl);
    REQUIRE(nwells >= 0 && (nwells == 0 || wells), "wells pointer required");
    {
        // the kernels address the Jacobian values with 32-bit integers: bound
        // nnzb*nb*nb from the dimensions before any per-cell array is read
        const long faces = (long)(grid->nx - 1) * grid->ny * grid->nz +
                           (long)grid->nx * (grid->ny - 1) * grid->nz +
                           (long)grid->nx * grid->ny * (grid->nz - 1);
        long nperf = 0;
        for (int wl = 0; wl < nwells; ++wl) nperf += std::max(wells[wl].nperf, 0);
        const long nbb = (fl && fl->model == FIM_BLACKOIL_3P) ? 9 : 4;
        const long nnzb = nl + 2 * faces + 2 * nperf + nwells;
        REQUIRE(nnzb * nbb < (1L << 31),
                "system too large: %ld blocks of %ld values (at most 2^31 - 1 values)", nnzb, nbb);
    }
    REQUIRE(grid->dx && grid->dy && grid->dz, "dx, dy, dz are required");
    for (int i = 0; i < grid->nx; ++i) REQUIRE(grid->dx[i] > 0, "dx must be > 0");
    for (int i = 0; i < grid->ny; ++i) REQUIRE(grid->dy[i] > 0, "dy must be > 0");
    for (int i = 0; i < grid->nz; ++i) REQUIRE(grid->dz[i] > 0, "dz must be > 0");
    REQUIRE(rock->kx && rock->ky && rock->kz && rock->poro, "rock arrays are required");
    for (long c = 0; c < nl; ++c) {
        REQUIRE(rock->kx[c] >= 0 && rock->ky[c] >= 0 && rock->kz[c] >= 0,
                "permeability must be >= 0 (cell %ld)", c);
        REQUIRE(rock->poro[c] > 0 && rock->poro[c] <= 1, "porosity must be in (0, 1] (cell %ld)", c);
    }
    REQUIRE(fl->model == FIM_DEADOIL_OW || fl->model == FIM_BLACKOIL_3P, "model must be 2 or 3");
    REQUIRE(fl->nrows >= 2 && fl->nrows <= kMaxTableRows, "PVT rows must be in [2, %d]",
            kMaxTableRows);
    REQUIRE(fl->p && fl->bo && fl->muo, "PVT columns p, bo, muo are required");
    const bool bo3 = fl->model == FIM_BLACKOIL_3P;
    if (bo3) REQUIRE(fl->rs && fl->bg && fl->mug, "model 3 needs rs, bg, mug columns");
    for (int r = 0; r < fl->nrows; ++r) {
        REQUIRE(fl->bo[r] > 0 && fl->muo[r] > 0, "Bo and muo must be > 0");
        if (bo3) REQUIRE(fl->bg[r] > 0 && fl->mug[r] > 0, "Bg and mug must be > 0");
        if (r + 1 < fl->nrows) {
            REQUIRE(fl->p[r + 1] > fl->p[r], "table pressures must increase");
            if (bo3) {
                REQUIRE(fl->rs[r + 1] > fl->rs[r], "Rs column must increase");
                const double dp = fl->p[r + 1] - fl->p[r];
                const double dRs = (fl->rs[r + 1] - fl->rs[r]) / dp;
                const double dBo = (fl->bo[r + 1] - fl->bo[r]) / dp;
                REQUIRE(fl->bg[r] * dRs > dBo,
                        "saturated row %d has negative total compressibility (Bg dRs/dP <= dBo/dP)", r);
            }
        }
    }
    REQUIRE(fl->bw_ref > 0 && fl->muw > 0, "water Bw_ref and muw must be > 0");
    REQUIRE(fl->swc >= 0 && fl->sor >= 0 && fl->sgc >= 0 &&
                fl->swc + fl->sor + (bo3 ? fl->sgc : 0.0) < 1,
            "end points must satisfy swc + sor (+ sgc) < 1");
    check_options(opt);

    auto *c = new fim_ctx();
    try {
        c->user_s = static_cast<hipStream_t>(stream);
        c->opt = *opt;
        c->g = Grid{grid->nx, grid->ny, grid->nz, (int)nl};
        c->n = (int)nl;
        c->nb = fl->model;
        c->nw = nwells;

        // wells: perforations sorted by cell within each well
        std::vector<int> sorted_cells;
        std::vector<double> wi_sorted, wi_dk_h, rw(nwells), skin(nwells);
        c->wps.assign(nwells + 1, 0);
        std::vector<int> pwell_h;
        int src_base = 0;
        for (int wl = 0; wl < nwells; ++wl) {
            const fim_well &W = wells[wl];
            REQUIRE(W.kind >= FIM_PROD && W.kind <= FIM_INJ_GAS, "well %d: bad kind", wl);
            REQUIRE(W.control == FIM_BHP || W.control == FIM_RATE, "well %d: bad control", wl);
            REQUIRE(!(W.kind == FIM_PROD && W.control == FIM_RATE),
                    "well %d: rate-controlled producers are not supported", wl);
            REQUIRE(!(W.kind == FIM_INJ_GAS && !bo3), "well %d: gas injection needs model 3", wl);
            REQUIRE(W.control == FIM_BHP || W.target > 0, "well %d: rate target must be > 0", wl);
            REQUIRE(W.nperf >= 1 && W.cells, "well %d: needs perforations", wl);
            REQUIRE(W.wi || W.rw > 0, "well %d: rw must be > 0 without explicit WI", wl);
            std::vector<int> idx(W.nperf);
            std::iota(idx.begin(), idx.end(), 0);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int a, int b2) { return W.cells[a] < W.cells[b2]; });
            for (int q = 0; q < W.nperf; ++q) {
                const int cell = W.cells[idx[q]];
                REQUIRE(cell >= 0 && cell < c->n, "well %d: perforation cell %d out of range", wl,
                        cell);
                REQUIRE(q == 0 || W.cells[idx[q - 1]] != cell, "well %d: duplicate cell %d", wl,
                        cell);
                sorted_cells.push_back(cell);
                pwell_h.push_back(wl);
                c->perf_src.push_back(src_base + idx[q]);
                wi_sorted.push_back(W.wi ? W.wi[idx[q]] : 0.0);
                wi_dk_h.push_back(W.wi ? 0.0 : 1.0);
                if (W.wi) REQUIRE(W.wi[idx[q]] > 0, "well %d: explicit WI must be > 0", wl);
            }
            src_base += W.nperf;
            c->wps[wl + 1] = c->wps[wl] + W.nperf;
            c->wkind.push_back(W.kind);
            c->wctrl.push_back(W.control);
            c->wtarget.push_back(W.target);
            rw[wl] = W.rw;
            skin[wl] = W.skin;
        }
        c->nperf = c->wps[nwells];
        c->nrows = c->n + nwells;
        c->nvec = (long)c->nrows * c->nb;

        // perforations of each cell in ascending well order
        std::vector<std::vector<int>> cell_wells(c->n);
        std::vector<int> cps(c->n + 1, 0), cperf;
        {
            std::vector<std::vector<int>> cell_perfs(c->n);
            for (int p = 0; p < c->nperf; ++p) {
                cell_wells[sorted_cells[p]].push_back(pwell_h[p]);
                cell_perfs[sorted_cells[p]].push_back(p);
            }
            for (int cell = 0; cell < c->n; ++cell) {
                cps[cell + 1] = cps[cell] + (int)cell_perfs[cell].size();
                for (int p : cell_perfs[cell]) cperf.push_back(p);
            }
        }
        std::vector<int> rp, ci, dp;
        build_pattern(c, rp, ci, dp, cell_wells, sorted_cells);
        c->nnzb = (int)ci.size();

        // fluid and rock scalars
        Phys &f = c->phys;
        f.model = fl->model;
        f.nrows = fl->nrows;
        f.co_us = fl->co_us;
        f.cmu_us = fl->cmu_us;
        f.bw_ref = fl->bw_ref;
        f.cw = fl->cw;
        f.muw = fl->muw;
        f.pw_ref = fl->pw_ref;
        f.rho_w = fl->rho_sc[0];
        f.rho_o = fl->rho_sc[1];
        f.rho_g = fl->rho_sc[2];
        f.swc = fl->swc;
        f.sor = fl->sor;
        f.sgc = fl->sgc;
        f.nw = fl->nw;
        f.no = fl->no;
        f.ng = fl->ng;
        f.krw_max = fl->krw_max;
        f.kro_max = fl->kro_max;
        f.krg_max = fl->krg_max;
        f.cr = rock->cr;
        f.pref = rock->pref;
        std::vector<double> tab(6 * fl->nrows, 1.0);
        for (int r = 0; r < fl->nrows; ++r) {
            tab[r] = fl->p[r];
            tab[fl->nrows + r] = fl->bo[r];
            tab[2 * fl->nrows + r] = bo3 ? fl->rs[r] : 0.0;
            tab[3 * fl->nrows + r] = fl->muo[r];
            tab[4 * fl->nrows + r] = bo3 ? fl->bg[r] : 1.0;
            tab[5 * fl->nrows + r] = bo3 ? fl->mug[r] : 1.0;
        }

        // device memory (everything above validated the input without the device)
        HIPCHECK(hipGetDevice(&c->dev));
        HIPCHECK(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking));
        HIPCHECK(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
        HIPCHECK(hipEventRecord(c->ev_user, c->user_s));
        HIPCHECK(hipStreamWaitEvent(c->s, c->ev_user, 0));
        const int n = c->n;
        c->dx = c->upload(grid->dx, grid->nx);
        c->dy = c->upload(grid->dy, grid->ny);
        c->dz = c->upload(grid->dz, grid->nz);
        c->kx = c->upload(rock->kx, n);
        c->ky = c->upload(rock->ky, n);
        c->kz = c->upload(rock->kz, n);
        c->poro = c->upload(rock->poro, n);
        c->tab = c->upload(tab.data(), tab.size());
        f.tab = c->tab;
        c->vol = c->alloc<double>(n);
        c->depth = c->alloc<double>(n);
        c->pvref = c->alloc<double>(n);
        c->tx = c->alloc<double>(n);
        c->ty = c->alloc<double>(n);
        c->tz = c->alloc<double>(n);
        c->dwkind = c->upload(c->wkind.data(), nwells);
        c->dwctrl = c->upload(c->wctrl.data(), nwells);
        c->dwtarget = c->upload(c->wtarget.data(), nwells);
        c->dwps = c->upload(c->wps.data(), nwells + 1);
        c->pcell = c->upload(sorted_cells.data(), c->nperf);
        c->pwell = c->upload(pwell_h.data(), c->nperf);
        c->wi = c->upload(wi_sorted.data(), c->nperf);
        c->wi_explicit = wi_sorted;
        c->top = grid->top;
        c->wi_dk = c->upload(wi_dk_h.data(), c->nperf);
        c->wrw = c->upload(rw.data(), nwells);
        c->wskin = c->upload(skin.data(), nwells);
        c->cps = c->upload(cps.data(), n + 1);
        c->cperf = c->upload(cperf.data(), cperf.size());
        c->P = c->alloc<double>(n);
        c->Sw = c->alloc<double>(n);
        c->X = c->alloc<double>(n);
        c->flag = c->alloc<int8_t>(n);
        c->pbhp = c->alloc<double>(std::max(nwells, 1));
        for (int k = 0; k < 2; ++k) {
            c->sP[k] = c->alloc<double>(n);
            c->sSw[k] = c->alloc<double>(n);
            c->sX[k] = c->alloc<double>(n);
            c->sflag[k] = c->alloc<int8_t>(n);
            c->spb[k] = c->alloc<double>(std::max(nwells, 1));
        }
        const int nrec = (c->nb == 2) ? Rec<2>::NREC : Rec<3>::NREC;
        c->rec = c->alloc<double>((size_t)nrec * n);
        c->aold = c->alloc<double>((size_t)c->nb * n);
        c->wmeas = c->alloc<double>(std::max(nwells, 1));
        c->rowptr = c->upload(rp.data(), rp.size());
        c->colind = c->upload(ci.data(), ci.size());
        c->diagpos = c->upload(dp.data(), dp.size());
        c->val = c->alloc<double>((size_t)c->nnzb * c->nb * c->nb);
        c->R = c->alloc<double>(c->nvec);
        c->dinv = c->alloc<double>((size_t)c->nrows * c->nb * c->nb);
        c->bad = c->alloc<int>(1);
        c->w = c->alloc<double>(c->nvec);
        c->z = c->alloc<double>(c->nvec);
        c->x = c->alloc<double>(c->nvec);
        c->r = c->alloc<double>(c->nvec);
        c->t = c->alloc<double>(c->nvec);
        c->b = c->alloc<double>(c->nvec);
        c->tmp = c->alloc<double>(kMaxRestart + 2);
        c->ydev = c->alloc<double>(kMaxRestart + 2);
        c->reorth = c->alloc<int>(1);
        alloc_krylov(c, opt->restart);
        c->perf_cell_h = sorted_cells;
        build_amg(c, sorted_cells, pwell_h);
        {
            // the level-0 AMG entry of every column (colour-split cell or
            // well), so the second CPR stage gathers without the split map
            const AmgLevel &L0 = c->lv[0];
            std::vector<int> cs(ci.size());
            for (size_t q = 0; q < ci.size(); ++q) {
                const int col = ci[q];
                if (col >= c->n) {
                    cs[q] = 2 * L0.half + (col - c->n);
                    continue;
                }
                const int i = col % c->g.nx, j = (col / c->g.nx) % c->g.ny,
                          k = col / (c->g.nx * c->g.ny);
                const int cc = i + L0.nxp * (j + c->g.ny * k);
                cs[q] = (((i + j + k) & 1) ? L0.half : 0) + (cc >> 1);
            }
            c->colsplit = c->upload(cs.data(), cs.size());
            c->sync();
        }
        build_subcycle(c);
        build_ilu(c);
        ensure_mixed(c);
        const size_t np = (size_t)(kMaxRestart + 2) * 2048 + (size_t)2048 * 16;
        c->partials = c->alloc<double>(np);
        c->scal = c->alloc<double>(S_COUNT);
        HIPCHECK(hipMemsetAsync(c->reorth, 0, sizeof(int), c->s));
        c->pin_len = S_COUNT + (size_t)(kMaxRestart + 1) * (kMaxRestart + 2) + kMaxRestart + 2;
        HIPCHECK(hipHostMalloc((void **)&c->pin, c->pin_len * sizeof(double), hipHostMallocDefault));
        for (auto &e : c->ev) HIPCHECK(hipEventCreate(&e));
        for (auto &e : c->colev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));

        // static precompute (PreProcess / ROCK / AllWells setup)
        launch_static(c->s, c->g, c->dx, c->dy, c->dz, grid->top, c->kx, c->ky, c->kz, c->poro,
                      c->vol, c->depth, c->pvref, c->tx, c->ty, c->tz);
        launch_peaceman(c->s, c->g, c->nperf, c->pcell, c->pwell, c->dx, c->dy, c->dz, c->kx,
                        c->ky, c->wrw, c->wskin, c->wi);
        HIPCHECK(hipGetLastError());
        c->sync();
    } catch (...) {
        delete c;
        throw;
    }
    *out = c;
    return FIM_OK;
}

// ---------------------------------------------------------------------------
// small device helpers

static void props(fim_ctx *c, bool with_aold) {
    launch_props(c->s, c->nb, c->phys, c->n, c->pvref, c->P, c->Sw, c->X, c->flag, c->rec,
                 with_aold ? c->aold : nullptr);
}

static void assemble(fim_ctx *c, double dt) {
    launch_assemble(c->s, c->nb, c->g, c->phys, c->wells(), c->sys(), c->depth, c->tx, c->ty,
                    c->tz, c->P, c->pbhp, c->rec, c->aold, dt, c->wmeas);
    c->jac_ready = true;
    c->prec_ready = false;
}

static void d2h_scalars(fim_ctx *c, int first, int count) {
    HIPCHECK(hipMemcpyAsync(c->pin + first, c->scal + first, count * sizeof(double),
                            hipMemcpyDeviceToHost, c->s));
}

static void save_state(fim_ctx *c, int slot) {
    const size_t n = c->n;
    HIPCHECK(hipMemcpyAsync(c->sP[slot], c->P, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->sSw[slot], c->Sw, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->sX[slot], c->X, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->sflag[slot], c->flag, n, hipMemcpyDeviceToDevice, c->s));
    if (c->nw)
        HIPCHECK(hipMemcpyAsync(c->spb[slot], c->pbhp, c->nw * 8, hipMemcpyDeviceToDevice, c->s));
}

static void restore_state(fim_ctx *c, int slot) {
    const size_t n = c->n;
    HIPCHECK(hipMemcpyAsync(c->P, c->sP[slot], n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->Sw, c->sSw[slot], n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->X, c->sX[slot], n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->flag, c->sflag[slot], n, hipMemcpyDeviceToDevice, c->s));
    if (c->nw)
        HIPCHECK(hipMemcpyAsync(c->pbhp, c->spb[slot], c->nw * 8, hipMemcpyDeviceToDevice, c->s));
}

// One cycle of the pressure AMG on level l (right-hand side in lv[l].b,
// result in lv[l].x): red-black Gauss-Seidel with zero initial guess,
// coarse-grid correction(s), then smoothing that applies the pending
// correction while it reads.
// One AMG cycle from level l down (paper Sec. 5.1: the pressure stage of
// CPR).  With rec == nullptr the phases are launched, and the sub-cycle
// rooted at c->sub_root runs as one fused launch; otherwise the phases are
// recorded into *rec with levels relative to root.
static void amg_cycle(fim_ctx *c, int l, std::vector<int> *rec = nullptr, int root = 0) {
    const int L = (int)c->lv.size();
    if (!rec && l == c->sub_root) {
        launch_amg_subcycle(c->s, c->sub);
        HIPCHECK(hipGetLastError());           // e.g. an LDS request the device refuses
        return;
    }
    const int rl = l - root;
    if (l == L - 1) {
        if (rec) rec->push_back(amg_op(kOpCoarse, rl));
        else if (c->exact_on) exact_apply(c, c->lv[l]);
        else launch_amg_coarsest_solve(c->s, c->lv[l], c->Minv);
        return;
    }
    const AmgLevel &F = c->lv[l], &C = c->lv[l + 1];
    const int nu = c->opt.amg_sweeps > 0 ? c->opt.amg_sweeps : 1;
    // default: V at the finest level, W below (the finest level dominates the
    // cost of a visit, the coarse ones the convergence)
    const int cyc = c->opt.amg_cycle;
    int gamma = (cyc == 1 || (cyc == 0 && l == 0)) ? 1 : 2;
    if (cyc >= 16 && 2L * F.half + F.nw > cyc) gamma = 1;   // V above the size limit
    if (cyc <= -16) gamma = (l > 0 && 2L * F.half + F.nw > -(long)cyc) ? 2 : 1;  // V at and below
    if (l + 1 == L - 1) gamma = 1;             // the coarsest level is solved exactly
    auto sweep = [&](int color, int mode) {
        if (rec) rec->push_back(amg_op(kOpSweep, rl, color, mode));
        else launch_amg_sweep(c->s, F, C, color, mode);
    };
    // a launched well sweep is folded into the presmoothing or colour-1
    // sweep before it (which then reads the wells from the snapshot the
    // colour-0 sweep took); in one workgroup it stays a phase of its own,
    // which is cheaper there than the recomputation the folding needs
    auto wells = [&] {
        if (F.nw == 0) return;
        if (rec) rec->push_back(amg_op(kOpWells, rl));
    };
    for (int sw = 0; sw < nu; ++sw) {
        if (sw == 0) {                          // both colours from a zero iterate
            if (rec) rec->push_back(amg_op(kOpPresmooth, rl));
            else launch_amg_presmooth(c->s, F);
        } else {
            sweep(0, 0);
            sweep(1, 0);
        }
        wells();
    }
    for (int gv = 0; gv < gamma; ++gv) {
        if (rec) {
            if (gv > 0) rec->push_back(amg_op(kOpCorrect, rl));
            rec->push_back(amg_op(kOpRestrict, rl));
        } else {
            if (gv > 0) launch_amg_correct(c->s, F, C);
            const int sr = c->opt.amg_seg_rows;
            launch_amg_restrict(c->s, F, C, sr == 0 ? (long)kSegRowsDefault : (long)sr);
        }
        amg_cycle(c, l + 1, rec, root);
    }
    for (int sw = 0; sw < nu; ++sw) {
        sweep(0, sw == 0 ? (kCellsCorr | kWellsCorr) : 0);
        sweep(1, sw == 0 ? kWellsCorr : 0);
        wells();
    }
}

// Choose the root of the fused sub-cycle (the first level with at most
// amg_fused cells and wells) and record its phase list; a sub-cycle whose
// levels or phase list do not fit (kSubLevels, kSubOps, the LDS of one
// workgroup) moves the root one level coarser.
static void build_subcycle(fim_ctx *c) {
    c->sub_root = -1;
    const int L = (int)c->lv.size();
    // (a coarsest level solved by slabs is its own single-workgroup launch)
    if (L == 0 || c->opt.amg_fused < 0 || c->exact_on) return;
    const long limit = c->opt.amg_fused > 0 ? c->opt.amg_fused : kFusedCellsDefault;
    int root = 0;
    while (root < L && 2L * c->lv[root].half + c->lv[root].nw > limit) ++root;
    int dev = 0, lds_max = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    std::vector<int> ops;
    AmgSub sub{};
    for (; root < L; ++root) {
        if (L - root > kSubLevels) continue;
        ops.clear();
        amg_cycle(c, root, &ops, root);
        if ((int)ops.size() > kSubOps) continue;
        sub = AmgSub{};
        sub.nlev = L - root;
        long nd = 0, ni = 0;
        for (int k = 0; k <= sub.nlev; ++k) {
            // the entry past the coarsest is never dereferenced
            const AmgLevel &Lk = (k < sub.nlev) ? c->lv[root + k] : AmgLevel{};
            if (k < sub.nlev) sub.lv[k] = Lk;
            const long n = 2L * Lk.half + Lk.nw;
            int *o = sub.off[k];
            o[kSubX] = (int)nd;
            o[kSubB] = (int)(nd + n);
            o[kSubAcw] = (int)(nd + 2 * n);
            o[kSubAwc] = (int)(nd + 2 * n + Lk.nslot);
            nd += 2 * n + 2L * Lk.nslot;
            o[kSubCps] = (int)ni;
            o[kSubCslot] = (int)(ni + 2L * Lk.half + 1);
            o[kSubSwell] = o[kSubCslot] + Lk.nslot;
            o[kSubScell] = o[kSubSwell] + Lk.nslot;
            o[kSubSps] = o[kSubScell] + Lk.nslot;
            ni += 2L * Lk.half + 1 + 3L * Lk.nslot + Lk.nw + 1;
        }
        sub.rbufoff = (int)nd;                   // the root's 2*half fine residuals
        nd += 2L * sub.lv[0].half;
        sub.ldoubles = (int)nd;
        sub.opsoff = (int)ni;
        sub.nops = (int)ops.size();
        sub.minvoff = -1;
        for (int k = 0; k <= sub.nlev; ++k) sub.off[k][kSubA] = -1;
        if (amg_subcycle_lds(sub) > (size_t)lds_max) continue;
        // what still fits goes to LDS too: the dense coarsest inverse first,
        // then stencil coefficients from the coarser levels up
        auto try_add = [&](long ndoubles) {
            AmgSub t = sub;
            t.ldoubles = (int)(sub.ldoubles + ndoubles);
            if (amg_subcycle_lds(t) > (size_t)lds_max) return -1;
            const int at = sub.ldoubles;
            sub.ldoubles = t.ldoubles;
            return at;
        };
        {
            const AmgLevel &Lc = sub.lv[sub.nlev - 1];
            const long nc = 2L * Lc.half + Lc.nw;
            sub.minvoff = try_add(nc * nc);
        }
        for (int k = sub.nlev - 2; k >= 0; --k) {
            sub.off[k][kSubA] = try_add(14L * sub.lv[k].half);
            if (sub.off[k][kSubA] < 0) break;
        }
        break;
    }
    if (root >= L) return;
    if (!c->sub_ops) c->sub_ops = c->alloc<int>(kSubOps);
    HIPCHECK(hipMemcpyAsync(c->sub_ops, ops.data(), ops.size() * sizeof(int),
                            hipMemcpyHostToDevice, c->s));
    // The LDS image in HBM: the arrays of the sub-cycle's levels move into
    // one buffer laid out as the launch's LDS, and every kernel reads and
    // writes them there (the launch before writes the root's right-hand
    // side in place), so a launch stages them with one flat copy.  An
    // earlier image stays allocated: levels outside this one may still point
    // into it.
    const size_t bytes = amg_subcycle_lds(sub);
    char *img = c->alloc<char>(bytes);
    HIPCHECK(hipMemsetAsync(img, 0, bytes, c->s));
    double *imd = reinterpret_cast<double *>(img);
    int *imi = reinterpret_cast<int *>(imd + sub.ldoubles);
    auto move_d = [&](double *&p, int off, long count) {
        if (count > 0)
            HIPCHECK(hipMemcpyAsync(imd + off, p, count * 8, hipMemcpyDeviceToDevice, c->s));
        p = imd + off;
    };
    auto move_i = [&](const int *&p, int off, long count) {
        if (count > 0)
            HIPCHECK(hipMemcpyAsync(imi + off, p, count * 4, hipMemcpyDeviceToDevice, c->s));
        p = imi + off;
    };
    for (int k = 0; k < sub.nlev; ++k) {
        AmgLevel &Lk = c->lv[root + k];
        const int *o = sub.off[k];
        const long n = 2L * Lk.half + Lk.nw;
        move_d(Lk.x, o[kSubX], n);
        move_d(Lk.b, o[kSubB], n);
        move_d(Lk.acw, o[kSubAcw], Lk.nslot);
        move_d(Lk.awc, o[kSubAwc], Lk.nslot);
        if (o[kSubA] >= 0) move_d(Lk.a, o[kSubA], 14L * Lk.half);
        move_i(Lk.cps, o[kSubCps], 2L * Lk.half + 1);
        move_i(Lk.cslot, o[kSubCslot], Lk.nslot);
        move_i(Lk.swell, o[kSubSwell], Lk.nslot);
        move_i(Lk.scell, o[kSubScell], Lk.nslot);
        move_i(Lk.sps, o[kSubSps], Lk.nw + 1);
        sub.lv[k] = Lk;
    }
    if (sub.minvoff >= 0) {
        const AmgLevel &Lc = c->lv[L - 1];
        const long nc = 2L * Lc.half + Lc.nw;
        move_d(c->Minv, sub.minvoff, nc * nc);
    }
    HIPCHECK(hipMemcpyAsync(imi + sub.opsoff, ops.data(), ops.size() * sizeof(int),
                            hipMemcpyHostToDevice, c->s));
    c->sync();
    // the device's limit rather than this context's need: every context sets
    // the same value, so none lowers the limit another one launches under
    HIPCHECK(amg_subcycle_allow_lds((size_t)lds_max));
    sub.ops = c->sub_ops;
    sub.Minv = c->Minv;
    sub.img = reinterpret_cast<const uint4 *>(img);
    sub.img_n16 = (int)(bytes / 16);
    c->sub = sub;
    c->sub_root = root;
}

static bool uses_ilu(const fim_options &o) {
    return o.precond == FIM_PREC_ILU0 || o.precond == FIM_PREC_CPR_ILU0;
}
static bool uses_cpr(const fim_options &o) {
    return o.precond == FIM_PREC_CPR || o.precond == FIM_PREC_CPR_ILU0;
}

// Subdomains of block-Jacobi ILU(0): boxes of the option's size, each with
// the wells whose perforations all lie in it (the others stand alone).
static void build_ilu(fim_ctx *c) {
    if (!uses_ilu(c->opt)) return;
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz, n = c->n, nw = c->nw;
    int d[3] = {c->opt.tile_nx, c->opt.tile_ny, c->opt.tile_nz};
    const int gd[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) d[a] = std::min(d[a] > 0 ? d[a] : 8, gd[a]);
    if (c->lu && d[0] == c->ilu_dims[0] && d[1] == c->ilu_dims[1] && d[2] == c->ilu_dims[2]) return;
    IluTiles T{};
    T.tx = d[0];
    T.ty = d[1];
    T.tz = d[2];
    T.ntx = (nx + T.tx - 1) / T.tx;
    T.nty = (ny + T.ty - 1) / T.ty;
    T.ntz = (nz + T.tz - 1) / T.tz;
    const int ntiles = T.ntx * T.nty * T.ntz;
    std::vector<int> rtile(n + nw), twp(ntiles + 1, 0), tw, wlocal(nw, -1), single;
    for (int cell = 0; cell < n; ++cell) {
        const int i = cell % nx, j = (cell / nx) % ny, k = cell / (nx * ny);
        rtile[cell] = i / T.tx + T.ntx * (j / T.ty + T.nty * (k / T.tz));
    }
    std::vector<std::vector<int>> joined(ntiles);
    for (int w = 0; w < nw; ++w) {
        int t = -1;
        bool one = true;
        for (int p = c->wps[w]; p < c->wps[w + 1]; ++p) {
            const int tp = rtile[c->perf_cell_h[p]];
            if (t < 0) t = tp;
            else if (tp != t) one = false;
        }
        if (one && t >= 0) {
            rtile[n + w] = t;
            wlocal[w] = (int)joined[t].size();
            joined[t].push_back(w);
        } else {
            rtile[n + w] = ntiles + w;
            single.push_back(w);
        }
    }
    for (int t = 0; t < ntiles; ++t) {
        twp[t + 1] = twp[t] + (int)joined[t].size();
        tw.insert(tw.end(), joined[t].begin(), joined[t].end());
        T.maxwells = std::max(T.maxwells, (int)joined[t].size());
    }
    // sweep records for tiles whose pencils fit one workgroup
    T.psteps = T.tx + T.ty + T.tz - 2;
    T.prec = T.tx * T.ty * T.tz;
    T.nnzb = c->nnzb;
    // (byte offsets of the raw buffers over A and the factors stay below 2^31)
    T.poff = (T.tx * T.ty <= 256 && ilu_rank_ints(T) <= 4096 &&
              (double)c->nnzb * c->nb * c->nb * sizeof(double) < 2147483648.0)
                 ? ((long)c->nnzb * c->nb * c->nb + 3) / 4 * 4 : -1;
    int dev = 0, lds_max = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    REQUIRE(ilu_solve_lds(c->nb, T) <= (size_t)lds_max && ilu_factor_lds(c->nb, T) <= (size_t)lds_max,
            "ILU(0) tile %d x %d x %d needs %zu bytes of LDS (at most %d)", T.tx, T.ty, T.tz,
            std::max(ilu_solve_lds(c->nb, T), ilu_factor_lds(c->nb, T)), lds_max);
    T.rtile = c->upload(rtile.data(), rtile.size());
    T.twp = c->upload(twp.data(), twp.size());
    T.tw = c->upload(tw.data(), std::max<size_t>(tw.size(), 1));
    T.wlocal = c->upload(wlocal.data(), std::max<size_t>(wlocal.size(), 1));
    T.single = c->upload(single.data(), std::max<size_t>(single.size(), 1));
    T.nsingle = (int)single.size();
    c->sync();                                  // the host vectors above are temporaries
    HIPCHECK(ilu_allow_lds(c->nb, (size_t)lds_max));   // the device's limit, as above
    const size_t elems = ilu_factor_elems(c->nb, c->nnzb, T, sizeof(double));
    if (c->lu_elems < elems) {
        c->drop_graphs();                       // captured steps name the old buffers
        c->release(c->lu);
        c->release(c->lu32);
        c->lu32 = nullptr;
        c->lu32_elems = 0;
        c->lu = c->alloc<double>(elems);
        c->lu_elems = elems;
    }
    if (!c->ilu_bad) c->ilu_bad = c->alloc<int>(1);
    c->ilu = T;
    for (int a = 0; a < 3; ++a) c->ilu_dims[a] = d[a];
}

// Single-precision buffers of the mixed mode: the Jacobian, the Krylov basis
// and its preconditioned images, the ILU(0) factors and the pressure column.
static void ensure_mixed(fim_ctx *c) {
    c->mixed = c->opt.precision == FIM_MIXED;
    if (!c->mixed) return;
    const size_t bs = (size_t)c->nb * c->nb;
    if (!c->val32) {
        c->val32 = c->alloc<float>((size_t)c->nnzb * bs);
        c->w32 = c->alloc<float>(c->nvec);
        c->ap32 = c->alloc<float>((size_t)c->nnzb * c->nb);
    }
    const size_t e32 = ilu_factor_elems(c->nb, c->nnzb, c->ilu, sizeof(float));
    if (c->lu32_elems < e32) {
        c->drop_graphs();
        c->release(c->lu32);
        c->lu32 = c->alloc<float>(e32);
        c->lu32_elems = e32;
    }
    if (c->m32 < c->m) {
        c->release(c->V32);
        c->release(c->Z32);
        c->V32 = c->alloc<float>((size_t)(c->m + 1) * c->nvec);
        c->Z32 = c->alloc<float>((size_t)(c->m + 1) * c->nvec);
        c->m32 = c->m;
    }
}

// The second-stage setup (BJ inverses or ILU(0) factors) on a stream, and
// the AMG hierarchy's extraction and coarsening on the context's stream.
static void second_stage_setup(fim_ctx *c, hipStream_t ss) {
    if (c->mixed) {
        launch_to_float(ss, (long)c->nnzb * c->nb * c->nb, c->val, c->val32);
        launch_ilu_factor(ss, c->nb, c->g, c->ilu, c->sys(), c->lu32, c->ilu_bad);
    } else if (!uses_ilu(c->opt)) {
        launch_bj_setup(ss, c->nb, c->nrows, c->diagpos, c->val, c->dinv, c->bad);
    } else {
        launch_ilu_factor(ss, c->nb, c->g, c->ilu, c->sys(), c->lu, c->ilu_bad);
    }
}
static void amg_levels_setup(fim_ctx *c, bool transposed) {
    if (transposed)
        launch_cprT_extract(c->s, c->nb, c->lv[0], c->g, c->wells(), c->sys(), c->wq, c->ap);
    else if (c->mixed)
        launch_amg_extract(c->s, c->nb, c->lv[0], c->g, c->wells(), c->sys(), c->wq, c->ap32);
    else
        launch_amg_extract(c->s, c->nb, c->lv[0], c->g, c->wells(), c->sys(), c->wq, c->ap);
    for (size_t l = 1; l < c->lv.size(); ++l)
        launch_amg_coarsen(c->s, c->lv[l - 1], c->lv[l], c->cfs_ptr[l], c->cfs_idx[l]);
}

// With CPR the second stage is set up on the side stream while the coarsest
// level's solver is (the slab factorisation ends in single-workgroup
// kernels that leave most of the device free); the two read the Jacobian
// and write disjoint arrays.
static void prec_setup_cpr(fim_ctx *c, bool transposed) {
    amg_levels_setup(c, transposed);
    HIPCHECK(hipEventRecord(c->ev_fork, c->s));
    HIPCHECK(hipStreamWaitEvent(c->s2, c->ev_fork, 0));
    second_stage_setup(c, c->s2);
    coarsest_setup(c);
    HIPCHECK(hipEventRecord(c->ev_join, c->s2));
    HIPCHECK(hipStreamWaitEvent(c->s, c->ev_join, 0));
    c->prec_ready = true;
}

static void prec_setup(fim_ctx *c) {
    if (uses_cpr(c->opt)) {
        prec_setup_cpr(c, false);
        return;
    }
    second_stage_setup(c, c->s);
    c->prec_ready = true;
}

// Buffers of the Krylov solver in element type T (double, or float for the
// inner solves of the mixed mode).
template <class T>
struct Kry;
template <>
struct Kry<double> {
    static double *V(fim_ctx *c) { return c->V; }
    static double *Z(fim_ctx *c) { return c->Z; }
    static double *w(fim_ctx *c) { return c->w; }
    static const double *val(fim_ctx *c) { return c->val; }
    static const double *lu(fim_ctx *c) { return c->lu; }
    static const double *ap(fim_ctx *c) { return c->ap; }
};
template <>
struct Kry<float> {
    static float *V(fim_ctx *c) { return c->V32; }
    static float *Z(fim_ctx *c) { return c->Z32; }
    static float *w(fim_ctx *c) { return c->w32; }
    static const float *val(fim_ctx *c) { return c->val32; }
    static const float *lu(fim_ctx *c) { return c->lu32; }
    static const float *ap(fim_ctx *c) { return c->ap32; }
};

// z = M^-1 v.  With hptr set, v = w / *hptr is formed (and stored) first,
// as for a new Arnoldi vector; without it v = w (stored in v's precision
// when v is given).  WT / T: element types of w and of v, z.
template <class WT, class T>
static void precondition(fim_ctx *c, const WT *w, const double *hptr, T *v, T *z) {
    constexpr bool same = std::is_same<WT, T>::value;
    if (c->opt.precond == FIM_PREC_CPR_ILU0) {
        launch_cpr_restrict(c->s, c->nb, c->n, c->nw, c->lv[0], c->split0, w, hptr, v,
                            c->cpr_rw ? c->cpr_rw : c->wq);
        amg_cycle(c, 0);
        const T *rhs = v;
        if constexpr (same) {
            if (!v) rhs = w;
        }
        IluRhs<T, T> R{rhs, Kry<T>::ap(c), c->colsplit, c->split0, c->lv[0].x,
                       2 * c->lv[0].half, c->cpr_pw};
        R.nxp = c->lv[0].nxp;
        launch_ilu_solve(c->s, c->nb, c->g, c->ilu, c->sys(), Kry<T>::lu(c), R, z);
    } else if (c->opt.precond == FIM_PREC_ILU0) {
        const T *rhs = v;
        if (hptr) {
            launch_normalize(c->s, c->nvec, w, hptr, v);
        } else if constexpr (same) {
            rhs = w;
        } else {
            launch_to_float(c->s, c->nvec, w, v);
        }
        const IluRhs<T, T> R{rhs, nullptr, nullptr, nullptr, nullptr, 0};
        launch_ilu_solve(c->s, c->nb, c->g, c->ilu, c->sys(), Kry<T>::lu(c), R, z);
    } else {
        if constexpr (std::is_same<T, double>::value && same) {
            if (c->opt.precond == FIM_PREC_CPR) {
                launch_cpr_restrict(c->s, c->nb, c->n, c->nw, c->lv[0], c->split0, w, hptr, v,
                                    c->wq);
                amg_cycle(c, 0);
                launch_cpr_finish(c->s, c->nb, c->n, c->nw, c->lv[0], c->split0, c->colsplit,
                                  c->sys(), c->ap, hptr ? v : w, c->dinv, z);
            } else if (hptr) {
                launch_normalize_precond(c->s, c->nb, c->nrows, w, hptr, v, z, c->dinv);
            } else {
                launch_bj_apply(c->s, c->nb, c->nrows, c->dinv, w, z);
            }
        } else {
            throw std::logic_error("preconditioner not available in single precision");
        }
    }
}

// Whether the next solver SpMV stamps its start and end into a pair of
// events: every opt.profile-th one when profiling (a stamp costs the launch
// a wait of its own)
static bool next_spmv_stamped(fim_ctx *c, bool profile) {
    return profile && c->spmv_seq++ % c->opt.profile == 0;
}

// SpMV inside the solver (y = J x in T), stamped or not
template <class T>
static void solver_spmv(fim_ctx *c, const T *xin, T *yout, bool stamp) {
    if (stamp) {
        if (c->spmv_used + 2 > (int)c->spmv_ev.size()) {
            // pool full: drain it
            HIPCHECK(hipEventSynchronize(c->spmv_ev[c->spmv_used - 1]));
            for (int k = 0; k < c->spmv_used; k += 2) {
                float ms = 0;
                HIPCHECK(hipEventElapsedTime(&ms, c->spmv_ev[k], c->spmv_ev[k + 1]));
                c->spmv_ms += ms;
            }
            c->spmv_used = 0;
        }
        launch_spmv(c->s, c->nb, c->nrows, c->rowptr, c->colind, Kry<T>::val(c), xin, yout,
                    c->spmv_ev[c->spmv_used], c->spmv_ev[c->spmv_used + 1]);
        HIPCHECK(hipGetLastError());
        c->spmv_used += 2;
        c->spmv_calls += 1;
    } else {
        launch_spmv(c->s, c->nb, c->nrows, c->rowptr, c->colind, Kry<T>::val(c), xin, yout);
    }
}

static void drain_spmv_events(fim_ctx *c) {
    if (!c->spmv_used) return;
    HIPCHECK(hipEventSynchronize(c->spmv_ev[c->spmv_used - 1]));
    for (int k = 0; k < c->spmv_used; k += 2) {
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, c->spmv_ev[k], c->spmv_ev[k + 1]));
        c->spmv_ms += ms;
    }
    c->spmv_used = 0;
}

// ---------------------------------------------------------------------------
// Flexible GMRES (right preconditioning, the preconditioned vectors Z kept)
// with classical Gram-Schmidt (a second, DGKS-triggered pass optional).  Solves
// J x = b (b, x device vectors of the context), initial guess zero.  The host
// stays one Arnoldi step behind the device: step j+1 is queued before the
// Hessenberg column of step j is read.

// Arnoldi step j after its SpMV (w = J z_j): a classical Gram-Schmidt pass
// (and, with gs_refine = 1, a second one gated on the device), the new
// basis vector and its preconditioned image; the Hessenberg column also
// goes to pinned host memory.
template <class T>
static void arnoldi_rest(fim_ctx *c, int j) {
    const long nv = c->nvec;
    const int LD = kMaxRestart + 2;
    double *col = c->H + (size_t)j * LD;
    double *pinH = c->pin + S_COUNT;
    T *V = Kry<T>::V(c), *Z = Kry<T>::Z(c), *w = Kry<T>::w(c);
    const bool refine = c->opt.gs_refine > 0;
    // the finishing kernels store the column in pinned host memory as well
    // (a copy node at the end of the graph would cost a launch)
    double *mirror = pinH + (size_t)j * LD;
    launch_multidot(c->s, nv, j + 1, V, w, c->partials, col, nullptr);
    launch_update_norm(c->s, nv, j + 1, V, col, w, c->partials, col + j + 1, nullptr,
                       refine ? c->reorth : nullptr, nullptr, mirror);
    if (refine) {
        launch_multidot(c->s, nv, j + 1, V, w, c->partials, c->tmp, c->reorth);
        launch_update_norm(c->s, nv, j + 1, V, c->tmp, w, c->partials, col + j + 1, c->reorth,
                           nullptr, col, mirror);
    }
    precondition<T, T>(c, w, col + j + 1, V + (size_t)(j + 1) * nv, Z + (size_t)(j + 1) * nv);
}

// Arnoldi step j as a captured graph: with its SpMV (w = J z_j) or, when
// the SpMV was launched on its own (stamped), without it
template <class T>
static void arnoldi_graph(fim_ctx *c, int j, bool with_spmv) {
    hipGraphExec_t &ex = with_spmv ? c->step_full[j] : c->step_exec[j];
    if (!ex) {
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
        try {
            if (with_spmv) solver_spmv<T>(c, Kry<T>::Z(c) + (size_t)j * c->nvec, Kry<T>::w(c), false);
            arnoldi_rest<T>(c, j);
        } catch (...) {
            (void)hipStreamEndCapture(c->s, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHECK(hipStreamEndCapture(c->s, &graph));
        hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
    }
    HIPCHECK(hipGraphLaunch(ex, c->s));
}

// Linear tolerance of a Newton iteration: the fixed lin_rtol, or the
// Eisenstat-Walker choice 2 (gamma 0.9, alpha 2) kept in [lin_rtol, 1e-2]
// with its safeguard against dropping too fast.
struct Forcing {
    double rn_prev = -1.0, eta_prev = 1e-2;
    double next(const fim_options &o, double rn) {
        const double eta_max = 1e-2;
        double eta = eta_max;
        if (o.forcing && rn_prev > 0.0) {
            eta = 0.9 * (rn / rn_prev) * (rn / rn_prev);
            const double guard = 0.9 * eta_prev * eta_prev;
            if (guard > 0.1) eta = std::max(eta, guard);
        }
        if (!o.forcing) eta = o.lin_rtol;
        eta = std::min(std::max(eta, o.lin_rtol), std::max(eta_max, o.lin_rtol));
        rn_prev = rn;
        eta_prev = eta;
        return eta;
    }
};

// In the mixed mode (T = float) every restart cycle is a single-precision
// inner solve of J d = r / ||r|| and every restart an FP64 refinement step
// (x += d, r = b - J x with the FP64 Jacobian); a cycle stops once its
// estimate fell kInner below its start, the limit of single precision.
template <class T>
static int gmres_t(fim_ctx *c, const double *bvec, double *xvec, int max_it, double rtol,
                   bool profile, int *iters_out, double *relres_out, Forcing *forcing) {
    constexpr double kInner = std::is_same<T, float>::value ? 1e-5 : 0.0;
    T *V = Kry<T>::V(c), *Z = Kry<T>::Z(c), *w = Kry<T>::w(c);
    const int m = c->m;
    const long nv = c->nvec;
    const int LD = kMaxRestart + 2;          // stride of a Hessenberg column
    const double *pinH = c->pin + S_COUNT;    // pinned copies of the columns
    double *piny = c->pin + S_COUNT + (size_t)(kMaxRestart + 1) * LD;
    launch_scale_copy(c->s, nv, nullptr, 0.0, xvec);
    launch_norm2(c->s, nv, bvec, c->partials, c->scal + S_NORM);
    d2h_scalars(c, S_NORM, 2);
    c->sync();
    const double bnorm = c->pin[S_NORM + 1];
    *iters_out = 0;
    if (!(bnorm > 0.0)) {
        *relres_out = (bnorm == 0.0) ? 0.0 : NAN;
        return bnorm == 0.0 ? 0 : -1;
    }
    if (forcing) rtol = forcing->next(c->opt, bnorm);
    std::vector<double> Hh((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    hipEvent_t *colev = c->colev;
    const double *rvec = bvec;
    const double *beta_dev = c->scal + S_NORM + 1;
    double beta = bnorm;
    int total = 0, status = 1;
    double relres = 1.0;

    auto enqueue = [&](int j) {
        c->gs_vectors += j + 1;
        const bool stamp = next_spmv_stamped(c, profile);
        if (c->opt.graphs && !stamp) {
            arnoldi_graph<T>(c, j, true);
        } else {
            solver_spmv<T>(c, Z + (size_t)j * nv, w, stamp);
            if (c->opt.graphs) arnoldi_graph<T>(c, j, false);
            else arnoldi_rest<T>(c, j);
        }
        HIPCHECK(hipEventRecord(colev[j], c->s));
    };

    {
        for (;;) {
            precondition<double, T>(c, rvec, beta_dev, V, Z);
            const double stop = std::max(rtol * bnorm, kInner * beta);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0;
            enqueue(0);
            for (int j = 0;; ++j) {
                if (j + 1 < m && total + j + 1 < max_it) enqueue(j + 1);
                HIPCHECK(hipEventSynchronize(colev[j]));
                const double *h = pinH + (size_t)j * LD;
                for (int i = 0; i <= j + 1; ++i) Hh[(size_t)i * m + j] = h[i];
                for (int i = 0; i < j; ++i) {
                    const double a = Hh[(size_t)i * m + j], bq = Hh[(size_t)(i + 1) * m + j];
                    Hh[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
                    Hh[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bq;
                }
                const double a = Hh[(size_t)j * m + j], bq = Hh[(size_t)(j + 1) * m + j];
                const double den = std::hypot(a, bq);
                cs[j] = den > 0 ? a / den : 1.0;
                sn[j] = den > 0 ? bq / den : 0.0;
                Hh[(size_t)j * m + j] = den;
                Hh[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                k = j + 1;
                const bool breakdown = !(h[j + 1] > 0.0) || !std::isfinite(h[j + 1]);
                if (std::fabs(g[j + 1]) <= stop || k == m || total + k >= max_it ||
                    breakdown || !std::isfinite(g[j + 1]))
                    break;
            }
            total += k;
            // least squares: back substitution on the rotated Hessenberg matrix
            for (int i = k - 1; i >= 0; --i) {
                double sacc = g[i];
                for (int jj = i + 1; jj < k; ++jj) sacc -= Hh[(size_t)i * m + jj] * y[jj];
                y[i] = sacc / Hh[(size_t)i * m + i];
            }
            for (int i = 0; i < k; ++i) piny[i] = y[i];
            HIPCHECK(hipMemcpyAsync(c->ydev, piny, k * sizeof(double), hipMemcpyHostToDevice, c->s));
            launch_axpy_multi(c->s, nv, k, Z, c->ydev, xvec);
            launch_spmv(c->s, c->nb, c->nrows, c->rowptr, c->colind, c->val, xvec, c->t);
            launch_residual(c->s, nv, bvec, c->t, c->r, c->partials, c->scal + S_RES);
            d2h_scalars(c, S_RES, 2);
            c->sync();
            beta = c->pin[S_RES + 1];
            relres = beta / bnorm;
            if (relres <= rtol) {
                status = 0;
                break;
            }
            if (total >= max_it || !std::isfinite(relres)) break;
            rvec = c->r;
            beta_dev = c->scal + S_RES + 1;
        }
    }
    *iters_out = total;
    *relres_out = relres;
    return status;
}

static int gmres(fim_ctx *c, const double *bvec, double *xvec, int max_it, double rtol,
                 bool profile, int *iters_out, double *relres_out, Forcing *forcing = nullptr) {
    if (c->mixed)
        return gmres_t<float>(c, bvec, xvec, max_it, rtol, profile, iters_out, relres_out, forcing);
    return gmres_t<double>(c, bvec, xvec, max_it, rtol, profile, iters_out, relres_out, forcing);
}

// ---------------------------------------------------------------------------
// Newton iterations for one sub-step (Sec. 3.2.5): 1 when converged.

struct NewtonStats {
    int newton = 0, linear = 0;
    double cnv[3] = {0, 0, 0}, mb[3] = {0, 0, 0};
    double last_dp = 0, last_ds = 0, well_res = 0;
    double t_asm = 0, t_lin = 0, t_upd = 0;
};

static float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

// FIM_DEBUG=1 in the environment prints one line per Newton iteration
static bool debug_on() {
    static const int on = [] {
        const char *e = std::getenv("FIM_DEBUG");
        return (e && *e && *e != '0') ? 1 : 0;
    }();
    return on != 0;
}

static bool newton(fim_ctx *c, double dt, NewtonStats &st) {
    const fim_options &o = c->opt;
    const int nb = c->nb;
    double last_dp = INFINITY, last_ds = INFINITY, last_viol = 0.0;
    bool pending_update = false;
    Forcing forcing;
    for (int it = 0;; ++it) {
        HIPCHECK(hipEventRecord(c->ev[0], c->s));
        props(c, it == 0);
        assemble(c, dt);
        launch_conv(c->s, nb, c->n, c->nw, c->rec, c->R, c->wmeas, dt, c->partials,
                    conv_blocks(c->n), c->scal + S_CONV);
        HIPCHECK(hipEventRecord(c->ev[1], c->s));
        d2h_scalars(c, S_CONV, S_NORM - S_CONV);
        c->sync();
        if (pending_update) st.t_upd += elapsed(c->ev[2], c->ev[3]);
        st.t_asm += elapsed(c->ev[0], c->ev[1]);
        const double *sc = c->pin + S_CONV;
        if (it > 0) {
            last_dp = c->pin[S_UPD];
            last_ds = c->pin[S_UPD + 1];
            last_viol = c->pin[S_UPD + 2];
        }
        bool finite = std::isfinite(last_dp) || it == 0;
        bool conv = it > 0;
        for (int i = 0; i < nb; ++i) {
            st.cnv[i] = sc[i];
            st.mb[i] = dt * std::fabs(sc[nb + i]) / sc[2 * nb + i];
            finite = finite && std::isfinite(st.cnv[i]) && std::isfinite(st.mb[i]);
            conv = conv && st.cnv[i] <= o.tol_cnv && st.mb[i] <= o.tol_mb;
        }
        const double wmax = sc[3 * nb];
        st.last_dp = last_dp;
        st.last_ds = last_ds;
        st.well_res = wmax;
        finite = finite && std::isfinite(wmax);
        if (!finite) return false;
        conv = conv && wmax <= o.tol_well && last_dp <= o.tol_dp && last_ds <= o.tol_ds;
        if (debug_on())
            std::fprintf(stderr,
                         "[fim] dt %.4g it %d cnv %.2e %.2e mb %.2e %.2e well %.2e dp %.2e ds %.2e%s\n",
                         dt, it, st.cnv[0], st.cnv[1], st.mb[0], st.mb[1], wmax, last_dp, last_ds,
                         conv ? " converged" : "");
        // a converged iterate must be physical: a root with a saturation
        // outside [0, 1] (beyond kSatSlack) fails the solve like a
        // non-finite one
        if (conv) return last_viol <= kSatSlack;
        if (it >= o.max_newton) return false;

        prec_setup(c);
        int li = 0;
        double rr = 0;
        const int gs = gmres(c, c->R, c->x, o.max_lin, o.lin_rtol, o.profile != 0, &li, &rr,
                             &forcing);
        HIPCHECK(hipEventRecord(c->ev[2], c->s));
        HIPCHECK(hipEventSynchronize(c->ev[2]));
        st.t_lin += elapsed(c->ev[1], c->ev[2]);
        st.linear += li;
        st.newton += 1;
        if (debug_on()) std::fprintf(stderr, "[fim]   linear %d iterations relres %.2e\n", li, rr);
        if (gs != 0 && !(std::isfinite(rr) && rr < 1.0)) return false;
        launch_newton_update(c->s, nb, c->phys, c->n, c->nw, c->x, o.ds_max, o.dp_max, c->P,
                             c->Sw, c->X, c->flag, c->pbhp, c->partials, update_blocks(c->n),
                             c->scal + S_UPD);
        HIPCHECK(hipEventRecord(c->ev[3], c->s));
        pending_update = true;
    }
}

// on_accept (optional) runs after every accepted sub-step with its length,
// while the state is the sub-step's end state
static int step_impl(fim_ctx *c, double dt, fim_step_report *rep,
                     const std::function<void(double)> *on_accept = nullptr) {
    REQUIRE(dt > 0 && std::isfinite(dt), "dt must be > 0");
    if (!c->state_set) {
        set_err("state not set (call fim_set_state first)");
        throw StateError();
    }
    fim_step_report r{};
    c->spmv_ms = 0;
    c->spmv_calls = 0;
    c->gs_vectors = 0.0;
    c->spmv_used = 0;
    if (c->opt.profile && c->spmv_ev.empty()) {
        c->spmv_ev.resize(2048);
        for (auto &e : c->spmv_ev) HIPCHECK(hipEventCreate(&e));
    }
    save_state(c, 0);
    double remaining = dt, h = dt;
    int status = FIM_OK;
    NewtonStats st;
    while (remaining > 1e-12 * dt) {
        const double tdt = std::min(h, remaining);
        save_state(c, 1);
        if (newton(c, tdt, st)) {
            remaining -= tdt;
            if (r.nsub < FIM_MAX_SUB) r.dt_sub[r.nsub] = tdt;
            r.nsub++;
            if (on_accept) (*on_accept)(tdt);
        } else {
            restore_state(c, 1);
            r.cuts++;
            if (r.cuts > c->opt.max_cuts) {
                restore_state(c, 0);
                status = FIM_NOT_CONVERGED;
                break;
            }
            h = 0.5 * tdt;
        }
    }
    // step-start accumulation of the next step
    props(c, true);
    drain_spmv_events(c);
    c->sync();
    c->jac_ready = false;
    r.newton_iters = st.newton;
    r.linear_iters = st.linear;
    r.converged = status == FIM_OK;
    r.dt_done = status == FIM_OK ? dt : 0.0;
    for (int i = 0; i < 3; ++i) {
        r.cnv[i] = st.cnv[i];
        r.mb[i] = st.mb[i];
    }
    r.t_assemble = st.t_asm;
    r.t_linear = st.t_lin;
    r.t_update = st.t_upd;
    r.spmv_ms = c->spmv_ms;
    r.spmv_calls = c->spmv_calls;
    r.gs_vectors = c->gs_vectors;
    r.last_dp = st.last_dp;
    r.last_ds = st.last_ds;
    r.well_res = st.well_res;
    if (rep) *rep = r;
    return status;
}

// ---------------------------------------------------------------------------
// discrete adjoint of the backward-Euler system

// copy the current state to slot m of a checkpoint set (allocated on first
// use), or back
static void put_ckpt(fim_ctx *c, std::vector<fim_ctx::Ckpt> &set, size_t m) {
    const size_t n = c->n;
    while (set.size() <= m) {
        fim_ctx::Ckpt k{c->alloc<double>(n), c->alloc<double>(n), c->alloc<double>(n),
                        c->alloc<double>(std::max(c->nw, 1)), c->alloc<int8_t>(n)};
        set.push_back(k);
    }
    const fim_ctx::Ckpt &k = set[m];
    HIPCHECK(hipMemcpyAsync(k.P, c->P, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(k.Sw, c->Sw, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(k.X, c->X, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(k.flag, c->flag, n, hipMemcpyDeviceToDevice, c->s));
    if (c->nw) HIPCHECK(hipMemcpyAsync(k.pbhp, c->pbhp, c->nw * 8, hipMemcpyDeviceToDevice, c->s));
}

static void get_ckpt(fim_ctx *c, const std::vector<fim_ctx::Ckpt> &set, size_t m) {
    const size_t n = c->n;
    const fim_ctx::Ckpt &k = set[m];
    HIPCHECK(hipMemcpyAsync(c->P, k.P, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->Sw, k.Sw, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->X, k.X, n * 8, hipMemcpyDeviceToDevice, c->s));
    HIPCHECK(hipMemcpyAsync(c->flag, k.flag, n, hipMemcpyDeviceToDevice, c->s));
    if (c->nw) HIPCHECK(hipMemcpyAsync(c->pbhp, k.pbhp, c->nw * 8, hipMemcpyDeviceToDevice, c->s));
}

// The transpose permutation of the (structurally symmetric) pattern and the
// work arrays of the backward sweep, once per context.
static void ensure_adjoint(fim_ctx *c) {
    if (c->tperm) return;
    const int nr = c->nrows;
    std::vector<int> rp(nr + 1), ci(c->nnzb), perm(c->nnzb, -1);
    HIPCHECK(hipMemcpyAsync(rp.data(), c->rowptr, (nr + 1) * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPCHECK(hipMemcpyAsync(ci.data(), c->colind, c->nnzb * sizeof(int), hipMemcpyDeviceToHost, c->s));
    c->sync();
    for (int r = 0; r < nr; ++r)
        for (int q = rp[r]; q < rp[r + 1]; ++q) {
            const int col = ci[q];
            for (int t = rp[col]; t < rp[col + 1]; ++t)
                if (ci[t] == r) {
                    perm[q] = t;
                    break;
                }
            REQUIRE(perm[q] >= 0, "block (%d, %d) has no transposed partner", r, col);
        }
    c->tperm = c->upload(perm.data(), perm.size());
    c->valT = c->alloc<double>((size_t)c->nnzb * c->nb * c->nb);
    c->lam[0] = c->alloc<double>(c->nvec);
    c->lam[1] = c->alloc<double>(c->nvec);
    c->arhs = c->alloc<double>(c->nvec);
    c->grad = c->alloc<double>(c->n);
    c->objp = c->alloc<double>((size_t)std::max(c->nperf, 1) * (c->nb + 1));
    c->objw = c->alloc<double>(2 * std::max(c->nw, 1));
    std::vector<double> e0((size_t)c->n * c->nb, 0.0);
    for (int cell = 0; cell < c->n; ++cell) e0[(size_t)cell * c->nb] = 1.0;
    c->e0w = c->upload(e0.data(), e0.size());
    c->sync();
}

// Preconditioner of J^T (held in c->val): ILU(0) of J^T in the boxes, and the
// transposed CPR first stage (pressure component restricted, A_p^T by the
// aggregation AMG, prolongation by the quasi-IMPES weights).
static void adjoint_prec_setup(fim_ctx *c) { prec_setup_cpr(c, true); }

// Forward: nsteps time steps of fim_step.  Backward, over the accepted
// sub-steps m = M..1:
//   J_m^T lam_m = (1/dt_{m+1}) (dA(x_m)/dx_m)^T lam_{m+1} - (dJ/dx_m)^T
// (the first term absent for m = M, the second only where a schedule step
// ends), then grad += lam_m^T dR_m/dtheta (+ dJ/dtheta at schedule ends).
// The sweep needs every sub-step state x_m.  With every == 0 the forward run
// keeps all of them; with every = k >= 1 it keeps only the state at the start
// of every k-th schedule step, and the sweep recomputes each segment of k
// steps from its checkpoint before going backward through it (the replayed
// sub-steps are the recorded ones, so the states are bit for bit those of the
// forward run and the gradient does not depend on k).
// The transposed systems are solved by FGMRES in FP64 to a relative
// residual of 1e-12, preconditioned by CPR for J^T: the transposed pressure
// stage, then block-Jacobi ILU(0) of J^T.
static int adjoint_impl(fim_ctx *c, int nsteps, const double *dt, const double *qobs_h,
                        int every, double *grad_h, fim_adjoint_report *rep) {
    using clock = std::chrono::steady_clock;
    REQUIRE(nsteps >= 1, "nsteps must be >= 1");
    REQUIRE(dt && grad_h, "dt and grad are required");
    REQUIRE(qobs_h || c->nw == 0, "q_obs is required");
    REQUIRE(every >= 0, "checkpoint_every must be >= 0");
    if (!c->state_set) {
        set_err("state not set (call fim_set_state first)");
        throw StateError();
    }
    ensure_adjoint(c);
    fim_adjoint_report r{};
    const auto t0 = clock::now();
    std::vector<double> hsub;              // accepted sub-step lengths
    std::vector<int> send(1, -1);          // schedule step that ends at sub-step m, else -1
    std::vector<int> first(nsteps + 1, 0); // state index at the start of each schedule step
    const int nseg = every > 0 ? (nsteps + every - 1) / every : 1;
    const size_t end_slot = (size_t)nseg;  // (every > 0) the forward end state
    if (every == 0) put_ckpt(c, c->ckpt, 0);
    const std::function<void(double)> hook = [&](double h) {
        hsub.push_back(h);
        send.push_back(-1);
        if (every == 0) put_ckpt(c, c->ckpt, hsub.size());
    };
    auto back_to_start = [&] {
        if (every == 0) get_ckpt(c, c->ckpt, 0);
        else get_ckpt(c, c->seg, 0);
        props(c, true);
        c->sync();
    };
    for (int st = 0; st < nsteps; ++st) {
        first[st] = (int)hsub.size();
        if (every > 0 && st % every == 0) put_ckpt(c, c->seg, (size_t)(st / every));
        fim_step_report sr{};
        const int status = step_impl(c, dt[st], &sr, &hook);
        r.steps += status == FIM_OK;
        r.cuts += sr.cuts;
        r.newton_iters += sr.newton_iters;
        r.linear_iters += sr.linear_iters;
        if (status != FIM_OK) {
            back_to_start();
            r.substeps = (int)hsub.size();
            if (rep) *rep = r;
            return FIM_NOT_CONVERGED;
        }
        send.back() = st;
    }
    const int M = (int)hsub.size();
    first[nsteps] = M;
    if (every > 0) put_ckpt(c, c->seg, end_slot);
    c->sync();
    const auto t1 = clock::now();
    r.substeps = M;
    const size_t nq = (size_t)nsteps * c->nw;
    if (nq > c->qobs_len) {
        c->release(c->qobs);
        c->qobs = c->alloc<double>(nq);
        c->qobs_len = nq;
    }
    if (nq) HIPCHECK(hipMemcpyAsync(c->qobs, qobs_h, nq * 8, hipMemcpyHostToDevice, c->s));
    HIPCHECK(hipMemsetAsync(c->grad, 0, c->n * sizeof(double), c->s));
    // forward configuration (segment recomputation) and adjoint configuration
    // (the transposed solves: FP64, CPR for J^T with the ILU(0) second stage);
    // captured Arnoldi steps belong to one of them, so a switch drops them
    const fim_options saved = c->opt;
    const bool saved_mixed = c->mixed;
    auto to_forward = [&] {
        c->opt = saved;
        c->mixed = saved_mixed;
        c->cpr_rw = c->cpr_pw = nullptr;
        c->drop_graphs();
    };
    auto to_adjoint = [&] {
        c->opt.precond = FIM_PREC_CPR_ILU0;
        c->mixed = false;
        c->cpr_rw = c->e0w;
        c->cpr_pw = c->wq;
        c->drop_graphs();
    };
    std::vector<double> jw((size_t)nsteps * 2 * std::max(c->nw, 1), 0.0);
    int status = FIM_OK;
    double t_rec = 0.0;
    size_t held = every == 0 ? (size_t)M + 1 : end_slot + 1;
    try {
        to_adjoint();
        build_ilu(c);
        const int max_it = std::max(c->opt.max_lin, 1000);
        double *lam_next = nullptr;
        int cur = 0;
        for (int g = nseg - 1; g >= 0 && status == FIM_OK; --g) {
            const int s0 = every > 0 ? g * every : 0;
            const int s1 = every > 0 ? std::min(nsteps, s0 + every) : nsteps;
            const int m0 = first[s0], m1 = first[s1];
            if (every > 0) {
                // recompute the segment's sub-step states from its checkpoint
                const auto tr = clock::now();
                to_forward();
                get_ckpt(c, c->seg, (size_t)g);
                put_ckpt(c, c->ckpt, 0);
                for (int m = m0 + 1; m <= m1; ++m) {
                    NewtonStats ns;
                    if (!newton(c, hsub[m - 1], ns)) {
                        set_err("recomputing sub-step %d from the checkpoint of step %d failed", m,
                                s0);
                        throw StateError();
                    }
                    put_ckpt(c, c->ckpt, (size_t)(m - m0));
                }
                c->sync();
                held = std::max(held, end_slot + 1 + (size_t)(m1 - m0) + 1);
                to_adjoint();
                t_rec += std::chrono::duration<double, std::milli>(clock::now() - tr).count();
            }
            auto slot = [&](int m) { return (size_t)(every > 0 ? m - m0 : m); };
            for (int m = m1; m > m0; --m) {
                get_ckpt(c, c->ckpt, slot(m - 1));
                props(c, true);                         // A(x_{m-1})
                get_ckpt(c, c->ckpt, slot(m));
                props(c, false);
                assemble(c, hsub[m - 1]);               // J_m
                const int st = send[m];
                const double *objp = nullptr, *objw = nullptr;
                if (st >= 0 && c->nw) {
                    launch_adj_objective(c->s, c->nb, c->wells(), c->n, c->P, c->pbhp, c->rec,
                                         c->wi_dk, c->qobs + (size_t)st * c->nw, c->objp, c->objw);
                    HIPCHECK(hipMemcpyAsync(jw.data() + (size_t)st * 2 * c->nw, c->objw,
                                            2 * c->nw * 8, hipMemcpyDeviceToHost, c->s));
                    objp = c->objp;
                    objw = c->objw;
                }
                launch_adj_rhs(c->s, c->nb, c->wells(), c->n, c->rec, lam_next,
                               m < M ? 1.0 / hsub[m] : 0.0, objp, objw, c->arhs);
                launch_bsr_transpose(c->s, c->nb, c->nnzb, c->tperm, c->val, c->valT);
                std::swap(c->val, c->valT);
                double *lam = c->lam[cur];
                int li = 0;
                double rr = 0.0;
                int gs = 0;
                try {
                    adjoint_prec_setup(c);
                    gs = gmres_t<double>(c, c->arhs, lam, max_it, 1e-12, false, &li, &rr, nullptr);
                } catch (...) {
                    std::swap(c->val, c->valT);
                    throw;
                }
                std::swap(c->val, c->valT);
                r.adjoint_iters += li;
                r.adjoint_relres = std::max(r.adjoint_relres, rr);
                if (gs != 0) {
                    set_err("adjoint solve of sub-step %d did not converge (relative residual %.3g)",
                            m, rr);
                    status = FIM_NOT_CONVERGED;
                    break;
                }
                launch_adj_grad(c->s, c->nb, c->g, c->wells(), c->depth, c->tx, c->ty, c->tz,
                                c->kx, c->ky, c->kz, c->dx, c->dy, c->dz, c->P, c->pbhp, c->rec,
                                c->wi_dk, lam, objp, c->grad);
                lam_next = lam;
                cur ^= 1;
            }
        }
        if (status == FIM_OK)
            HIPCHECK(hipMemcpyAsync(grad_h, c->grad, c->n * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
    } catch (...) {
        to_forward();
        throw;
    }
    to_forward();
    // leave the context at the end of the forward run
    if (every == 0) get_ckpt(c, c->ckpt, (size_t)M);
    else get_ckpt(c, c->seg, end_slot);
    props(c, true);
    c->jac_ready = false;
    c->prec_ready = false;
    c->sync();
    for (int st = 0; st < nsteps; ++st)
        for (int wl = 0; wl < c->nw; ++wl) r.objective += jw[(size_t)st * 2 * c->nw + 2 * wl + 1];
    r.t_forward_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    r.t_adjoint_ms = std::chrono::duration<double, std::milli>(clock::now() - t1).count();
    r.t_recompute_ms = t_rec;
    r.stored_states = (int)held;
    if (rep) *rep = r;
    return status;
}

// ---------------------------------------------------------------------------
// batched ensemble: the members advanced together, one launch per kernel
// for all of them
//
// Every member keeps its own context (its buffers, options and schedule);
// a launch covers all members, each member's blocks running the member's
// own kernel bodies on the member's buffers, and per-member flags select
// the members that take part in it.  The host keeps the Newton / time-step
// state machine and the GMRES state of fim_step for every member, so a
// member computes bit for bit what it computes alone.  Newton iterations
// run in rounds: every member with work takes part in the round's
// assembly; the members whose convergence check asks for a solve share one
// lockstep FGMRES (restart cycles synchronised, a member frozen once its
// own cycle stops), then one update.

namespace {

struct Shape {                    // block starts of one launch shape
    int *d = nullptr;
    int total = 0;
};

enum { kSave0 = 128, kSave1 = 256, kRestore0 = 512, kRestore1 = 1024 };

// keys of the captured phases
enum { kPhaseAssemble = 1, kPhaseSetup, kPhaseGmresInit, kPhaseCycleStart, kPhaseFinish,
       kPhaseUpdate, kPhaseSave0, kPhaseSave1, kPhaseRestore0, kPhaseRestore1,
       kPhaseArnoldi = 100 };

struct GmState {
    bool in_cycle = false, stopped = false, first = true;
    int k = 0, total = 0, status = 1;
    double bnorm = 0, beta = 0, rtol = 0, stop = 0, relres = 1;
    std::vector<double> Hh, cs, sn, g, y;
};

struct MemRun {
    int st = 0;                   // schedule step
    bool stopped = false;         // no more work (all steps done, or one failed)
    double dt = 0, remaining = 0, h = 0, tdt = 0;
    int it = 0;
    double last_dp = INFINITY, last_ds = INFINITY, last_viol = 0;
    NewtonStats ns;
    fim_step_report rep{};
    Forcing forcing;
    bool start_step = true, start_sub = true, solve = false;
    GmState gm;
};

struct Ensemble {
    std::vector<fim_ctx *> mem;
    int nm = 0, nb = 0, m = 0, ilu_threads = 0, dense_n = 0;
    size_t exact_factor_lds = 0, exact_solve_lds = 0;   // members with a slab-solved level
    size_t ilu_lds = 0;
    hipStream_t s = nullptr;
    std::vector<void *> owned;
    Member *d_mem = nullptr;
    StateSlots *d_slots = nullptr;
    int *d_flags = nullptr, *d_k = nullptr;
    double *d_dt = nullptr, *d_scal = nullptr, *d_ypack = nullptr;
    int *h_flagring = nullptr;    // pinned ring of flag arrays
    int ring = 0, ringpos = 0;
    int *h_k = nullptr;
    double *h_dt = nullptr, *h_scal = nullptr, *h_ypack = nullptr;
    int ld_scal = 0, ld_y = 0;
    Shape cells, rows, wells, conv, one, vec, spmv, tiles, extract, statecopy;
    std::vector<Shape> coarsen, dot, dotsum;
    std::vector<int> flags;
    std::map<int, hipGraphExec_t> graphs;     // captured phases, by key
    bool use_graphs = true;
    bool refine = true;        // the Gram-Schmidt second pass when cancelled

    template <typename T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        if (count == 0) count = 1;
        const hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            set_err("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
            throw std::bad_alloc();
        }
        owned.push_back(p);
        return static_cast<T *>(p);
    }
    ~Ensemble() {
        if (s) (void)hipStreamSynchronize(s);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        for (void *p : owned) (void)hipFree(p);
        for (void *p : {(void *)h_flagring, (void *)h_k, (void *)h_dt, (void *)h_scal,
                        (void *)h_ypack})
            if (p) (void)hipHostFree(p);
        if (s) (void)hipStreamDestroy(s);
    }

    Shape shape(const std::function<int(const fim_ctx *)> &blocks) {
        std::vector<int> h(nm + 1, 0);
        for (int k = 0; k < nm; ++k) h[k + 1] = h[k] + std::max(0, blocks(mem[k]));
        Shape sh;
        sh.d = dalloc<int>(nm + 1);
        HIPCHECK(hipMemcpy(sh.d, h.data(), (nm + 1) * sizeof(int), hipMemcpyHostToDevice));
        sh.total = h[nm];
        return sh;
    }
    Batch batch(const Shape &sh, int bit) const { return Batch{sh.d, d_flags, nm, bit}; }

    // The launches of one phase: captured into a HIP graph on first use
    // (every argument, flags array included, is fixed per key: what changes
    // between rounds lives in device memory), then replayed.
    void phase(int key, const std::function<void()> &f) {
        if (!use_graphs) {
            f();
            return;
        }
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            hipGraph_t g = nullptr;
            HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                f();
            } catch (...) {
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIPCHECK(hipStreamEndCapture(s, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHECK(e);
            it = graphs.emplace(key, ex).first;
        }
        HIPCHECK(hipGraphLaunch(it->second, s));
    }

    // the host's flags to the device, in stream order (each copy from a
    // pinned ring slot of its own, so a later write does not race it)
    void put_flags() {
        int *slot = h_flagring + (size_t)ringpos * nm;
        ringpos = (ringpos + 1) % ring;
        if (ringpos == 0) HIPCHECK(hipStreamSynchronize(s));
        std::memcpy(slot, flags.data(), nm * sizeof(int));
        HIPCHECK(hipMemcpyAsync(d_flags, slot, nm * sizeof(int), hipMemcpyHostToDevice, s));
    }
    void set(int bit, const std::function<bool(int)> &on) {
        for (int k = 0; k < nm; ++k) flags[k] = on(k) ? (flags[k] | bit) : (flags[k] & ~bit);
    }
    bool any(int bit) const {
        for (int f : flags)
            if (f & bit) return true;
        return false;
    }
    // the members' scalar slots [first, first + count) into h_scal[k * ld_scal + e]
    // (queued; read after a synchronisation)
    void gather(int bit, int first, int count) {
        launchb_gather_scalars(s, d_mem, batch(one, bit), one.total, first, count, d_scal, ld_scal);
        HIPCHECK(hipMemcpyAsync(h_scal, d_scal, (size_t)nm * ld_scal * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    }
    void sync() { HIPCHECK(hipStreamSynchronize(s)); }
};

// the batched configuration: CPR with the block-Jacobi ILU(0) second stage
// in FP64, one block size, device, restart length and ILU(0) workgroup size
void check_member(const fim_ctx *c, const fim_ctx *c0, int k) {
    REQUIRE(c->opt.precond == FIM_PREC_CPR_ILU0 && c->opt.precision == FIM_FP64,
            "member %d: the batched ensemble runs CPR with block-Jacobi ILU(0) in FP64", k);
    REQUIRE(c->nb == c0->nb, "member %d: block size %d, member 0 has %d", k, c->nb, c0->nb);
    REQUIRE(c->dev == c0->dev, "member %d is on device %d, member 0 on %d", k, c->dev, c0->dev);
    REQUIRE(c->m == c0->m, "member %d: GMRES restart %d, member 0 has %d", k, c->m, c0->m);
    REQUIRE((c->opt.gs_refine > 0) == (c0->opt.gs_refine > 0),
            "member %d: Gram-Schmidt refinement differs from member 0's", k);
    REQUIRE(ilu_threads(c->ilu) == ilu_threads(c0->ilu),
            "member %d: ILU(0) boxes of %d threads, member 0's of %d", k, ilu_threads(c->ilu),
            ilu_threads(c0->ilu));
    REQUIRE((int)c->lv.size() < kMaxLevels, "member %d: %zu AMG levels (at most %d)", k,
            c->lv.size(), kMaxLevels - 1);
    const AmgLevel &Lc = c->lv.back();
    REQUIRE(c->exact_on || 2 * Lc.half + Lc.nw <= dense_lds_max(),
            "member %d: coarsest AMG level of %d entries (at most %d)", k, 2 * Lc.half + Lc.nw,
            dense_lds_max());
    if (!c->state_set) {
        set_err("member %d: state not set", k);
        throw StateError();
    }
}

std::unique_ptr<Ensemble> make_ensemble(int count, fim_ctx *const *members) {
    auto E = std::make_unique<Ensemble>();
    E->mem.assign(members, members + count);
    E->nm = count;
    E->flags.assign(count, 0);
    fim_ctx *c0 = members[0];
    for (int k = 0; k < count; ++k) check_member(members[k], c0, k);
    E->nb = c0->nb;
    E->m = c0->m;
    E->refine = c0->opt.gs_refine > 0;
    HIPCHECK(hipSetDevice(c0->dev));
    HIPCHECK(hipStreamCreateWithFlags(&E->s, hipStreamNonBlocking));
    for (fim_ctx *c : E->mem) c->sync();       // every member's earlier work is done
    int lds_max = 0;
    HIPCHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c0->dev));
    std::vector<Member> hm(count);
    std::vector<StateSlots> hs(count);
    for (int k = 0; k < count; ++k) {
        fim_ctx *c = members[k];
        Member &M = hm[k];
        std::memset(static_cast<void *>(&M), 0, sizeof M);
        M.g = c->g;
        M.f = c->phys;
        M.wells = c->wells();
        M.sys = c->sys();
        M.n = c->n;
        M.nw = c->nw;
        M.nb = c->nb;
        M.nrows = c->nrows;
        M.m = c->m;
        M.nvec = c->nvec;
        M.ds_max = c->opt.ds_max;
        M.dp_max = c->opt.dp_max;
        M.pvref = c->pvref;
        M.depth = c->depth;
        M.tx = c->tx;
        M.ty = c->ty;
        M.tz = c->tz;
        M.P = c->P;
        M.Sw = c->Sw;
        M.X = c->X;
        M.pbhp = c->pbhp;
        M.flag = c->flag;
        M.rec = c->rec;
        M.aold = c->aold;
        M.wmeas = c->wmeas;
        M.partials = c->partials;
        M.scal = c->scal;
        M.V = c->V;
        M.Z = c->Z;
        M.w = c->w;
        M.x = c->x;
        M.b = c->b;
        M.r = c->r;
        M.t = c->t;
        M.H = c->H;
        M.tmp = c->tmp;
        M.ydev = c->ydev;
        M.reorth = c->reorth;
        M.T = c->ilu;
        M.lu = c->lu;
        M.ilu_bad = c->ilu_bad;
        M.nlev = (int)c->lv.size();
        for (int l = 0; l < M.nlev; ++l) {
            M.lv[l] = c->lv[l];
            M.cfs_ptr[l] = c->cfs_ptr[l];
            M.cfs_idx[l] = c->cfs_idx[l];
        }
        M.split0 = c->split0;
        M.colsplit = c->colsplit;
        M.wq = c->wq;
        M.ap = c->ap;
        M.Mden = c->Mden;
        M.Minv = c->Minv;
        M.colk = c->colk;
        M.amg_bad = c->amg_bad;
        M.exact = c->exact_on ? 1 : 0;
        M.ex = c->ex;
        // the member's whole cycle from its finest level, and the
        // restriction's scratch
        std::vector<int> ops;
        amg_cycle(c, 0, &ops, 0);
        int *dops = E->dalloc<int>(ops.size());
        HIPCHECK(hipMemcpy(dops, ops.data(), ops.size() * sizeof(int), hipMemcpyHostToDevice));
        M.ops = dops;
        M.nops = (int)ops.size();
        M.rbuf = E->dalloc<double>(2 * (size_t)c->lv[0].half);
        for (int q = 0; q < 2; ++q) {
            hs[k].P[q] = c->sP[q];
            hs[k].Sw[q] = c->sSw[q];
            hs[k].X[q] = c->sX[q];
            hs[k].pbhp[q] = c->spb[q];
            hs[k].flag[q] = c->sflag[q];
        }
        E->ilu_lds = std::max({E->ilu_lds, ilu_solve_lds(c->nb, c->ilu), ilu_factor_lds(c->nb, c->ilu)});
        const AmgLevel &Lc = c->lv.back();
        if (c->exact_on) {
            E->exact_factor_lds = std::max(E->exact_factor_lds, exact_factor_lds(c->ex));
            E->exact_solve_lds = std::max(E->exact_solve_lds, exact_solve_lds(c->ex));
        } else {
            E->dense_n = std::max(E->dense_n, 2 * Lc.half + Lc.nw);
        }
    }
    REQUIRE(E->ilu_lds <= (size_t)lds_max, "ILU(0) boxes need %zu bytes of LDS (at most %d)",
            E->ilu_lds, lds_max);
    E->ilu_threads = ilu_threads(c0->ilu);
    HIPCHECK(ilu_batch_allow_lds(E->nb, (size_t)lds_max));
    HIPCHECK(batch_allow_lds());
    E->d_mem = E->dalloc<Member>(count);
    HIPCHECK(hipMemcpy(E->d_mem, hm.data(), count * sizeof(Member), hipMemcpyHostToDevice));
    E->d_slots = E->dalloc<StateSlots>(count);
    HIPCHECK(hipMemcpy(E->d_slots, hs.data(), count * sizeof(StateSlots), hipMemcpyHostToDevice));
    E->d_flags = E->dalloc<int>(count);
    E->d_k = E->dalloc<int>(count);
    E->d_dt = E->dalloc<double>(count);
    E->ld_scal = S_NORM + 4;
    E->ld_y = kMaxRestart + 2;
    E->d_scal = E->dalloc<double>((size_t)count * E->ld_scal);
    E->d_ypack = E->dalloc<double>((size_t)count * E->ld_y);
    E->ring = 4 * (kMaxRestart + 8);
    HIPCHECK(hipHostMalloc((void **)&E->h_flagring, (size_t)E->ring * count * sizeof(int),
                           hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void **)&E->h_k, count * sizeof(int), hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void **)&E->h_dt, count * sizeof(double), hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void **)&E->h_scal, (size_t)count * E->ld_scal * sizeof(double),
                           hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void **)&E->h_ypack, (size_t)count * E->ld_y * sizeof(double),
                           hipHostMallocDefault));
    // launch shapes: the block counts of the single-member launches
    E->cells = E->shape([](const fim_ctx *c) { return blocks_for_cells(c->n); });
    E->rows = E->shape([](const fim_ctx *c) { return blocks_for_cells(c->nrows); });
    E->statecopy = E->shape([](const fim_ctx *c) { return blocks_for_cells(std::max(c->n, c->nw)); });
    E->wells = E->shape([](const fim_ctx *c) { return c->nw; });
    E->conv = E->shape([](const fim_ctx *c) { return conv_blocks(c->n); });
    E->one = E->shape([](const fim_ctx *) { return 1; });
    E->vec = E->shape([](const fim_ctx *c) { return vec_blocks(c->nvec); });
    E->spmv = E->shape([](const fim_ctx *c) { return spmv_blocks(c->nb, c->nrows); });
    E->tiles = E->shape([](const fim_ctx *c) {
        return c->ilu.ntx * c->ilu.nty * c->ilu.ntz + (c->ilu.nsingle > 0 ? 1 : 0);
    });
    E->extract = E->shape([](const fim_ctx *c) {
        return (int)((8L * (c->n + c->nw) + kBlock - 1) / kBlock);
    });
    int maxlev = 0;
    for (fim_ctx *c : E->mem) maxlev = std::max(maxlev, (int)c->lv.size());
    E->coarsen.resize(maxlev);
    for (int l = 1; l < maxlev; ++l)
        E->coarsen[l] = E->shape([l](const fim_ctx *c) {
            if (l >= (int)c->lv.size()) return 0;
            const AmgLevel &C = c->lv[l];
            return (int)((2L * C.half + C.nslot + C.nw + kBlock - 1) / kBlock);
        });
    const int maxg = dot_groups(E->m);
    E->dot.resize(maxg + 1);
    for (int g = 1; g <= maxg; ++g)
        E->dot[g] = E->shape([g](const fim_ctx *c) { return vec_blocks(c->nvec) * g; });
    E->dotsum.resize(E->m + 1);
    for (int j = 0; j < E->m; ++j)
        E->dotsum[j] = E->shape([j](const fim_ctx *) { return j + 2; });
    return E;
}

// The preconditioner of every member with kOnSolve (prec_setup in FP64 with
// CPR and block-Jacobi ILU(0))
void batch_prec_setup(Ensemble &E) {
    launchb_ilu_factor(E.s, E.nb, E.d_mem, E.batch(E.tiles, kOnSolve), E.tiles.total,
                       E.ilu_threads, E.ilu_lds);
    launchb_amg_extract(E.s, E.nb, E.d_mem, E.batch(E.extract, kOnSolve), E.extract.total);
    for (size_t l = 1; l < E.coarsen.size(); ++l)
        launchb_amg_coarsen(E.s, E.d_mem, E.batch(E.coarsen[l], kOnSolve), E.coarsen[l].total,
                            (int)l);
    launchb_amg_coarsest(E.s, E.d_mem, E.batch(E.one, kOnSolve), E.one.total, E.dense_n,
                         E.exact_factor_lds);
}

// z = M^-1 v of the members with kOnCycle: the first vector of a restart
// cycle (j < 0) or the new Arnoldi vector of step j
void batch_precondition(Ensemble &E, int j) {
    launchb_cpr_restrict(E.s, E.nb, E.d_mem, E.batch(E.rows, kOnCycle), E.rows.total, j,
                         kFirstCycle, S_NORM, S_RES);
    launchb_amg_cycle(E.s, E.d_mem, E.batch(E.one, kOnCycle), E.one.total, E.exact_solve_lds);
    launchb_ilu_solve(E.s, E.nb, E.d_mem, E.batch(E.tiles, kOnCycle), E.tiles.total, j,
                      E.ilu_threads, E.ilu_lds);
}

// Arnoldi step j of the members with kOnCycle (arnoldi_rest after the SpMV),
// the Hessenberg columns packed into d_scal... into d_ypack's neighbour
void batch_arnoldi(Ensemble &E, int j, double *dcols, double *hcols, int ld) {
    launchb_spmv(E.s, E.nb, E.d_mem, E.batch(E.spmv, kOnCycle), E.spmv.total, j);
    const Shape &dp = E.dot[dot_groups(j + 1)];
    launchb_multidot(E.s, E.d_mem, E.batch(dp, kOnCycle), dp.total, E.batch(E.dotsum[j], kOnCycle),
                     E.dotsum[j].total, j, false);
    launchb_update_norm(E.s, E.d_mem, E.batch(E.vec, kOnCycle), E.vec.total,
                        E.batch(E.one, kOnCycle), E.one.total, j, false);
    if (E.refine) {
        launchb_multidot(E.s, E.d_mem, E.batch(dp, kOnCycle), dp.total,
                         E.batch(E.dotsum[j], kOnCycle), E.dotsum[j].total, j, true);
        launchb_update_norm(E.s, E.d_mem, E.batch(E.vec, kOnCycle), E.vec.total,
                            E.batch(E.one, kOnCycle), E.one.total, j, true);
    }
    batch_precondition(E, j);
    launchb_hcols(E.s, E.d_mem, E.batch(E.one, kOnCycle), E.one.total, j, dcols, ld);
    HIPCHECK(hipMemcpyAsync(hcols, dcols, (size_t)E.nm * ld * sizeof(double),
                            hipMemcpyDeviceToHost, E.s));
}

}  // namespace

namespace {

// FGMRES of the members with solve set (J x = R of each member, lin_rtol or
// its forcing term, max_lin iterations): gmres_t<double> of every member,
// with the restart cycles in lockstep.  Fills gm.status / total / relres.
void batch_gmres(Ensemble &E, std::vector<MemRun> &runs, double *dcols, double *hcols) {
    const int nm = E.nm, m = E.m, LDH = kMaxRestart + 2;
    const size_t colstride = (size_t)nm * LDH;       // one step's packed columns
    E.set(kOnSolve, [&](int k) { return runs[k].solve; });
    E.set(kOnCycle | kOnFinish | kFirstCycle, [](int) { return false; });
    E.put_flags();
    E.phase(kPhaseGmresInit, [&] {
        launchb_scale_zero(E.s, E.d_mem, E.batch(E.vec, kOnSolve), E.vec.total);
        launchb_norm_b(E.s, E.d_mem, E.batch(E.vec, kOnSolve), E.vec.total,
                       E.batch(E.one, kOnSolve), E.one.total, S_NORM);
        E.gather(kOnSolve, S_NORM, 2);
    });
    E.sync();
    for (int k = 0; k < nm; ++k) {
        MemRun &R = runs[k];
        if (!R.solve) continue;
        GmState &G = R.gm;
        fim_ctx *c = E.mem[k];
        G = GmState{};
        G.bnorm = E.h_scal[(size_t)k * E.ld_scal + 1];
        G.Hh.assign((size_t)(m + 1) * m, 0.0);
        G.cs.assign(m, 0.0);
        G.sn.assign(m, 0.0);
        G.g.assign(m + 1, 0.0);
        G.y.assign(m, 0.0);
        if (!(G.bnorm > 0.0)) {                // zero right side, or not a number
            G.relres = G.bnorm == 0.0 ? 0.0 : NAN;
            G.status = G.bnorm == 0.0 ? 0 : -1;
            continue;
        }
        G.rtol = R.forcing.next(c->opt, G.bnorm);
        G.beta = G.bnorm;
        G.in_cycle = true;
        G.first = true;
    }
    for (;;) {
        // one restart cycle of the members still solving
        bool anyc = false;
        for (int k = 0; k < nm; ++k) {
            GmState &G = runs[k].gm;
            if (!runs[k].solve || !G.in_cycle) continue;
            anyc = true;
            G.stopped = false;
            G.k = 0;
            G.stop = G.rtol * G.bnorm;
            std::fill(G.g.begin(), G.g.end(), 0.0);
            G.g[0] = G.beta;
        }
        if (!anyc) break;
        auto cycle_member = [&](int k) { return runs[k].solve && runs[k].gm.in_cycle; };
        E.set(kOnCycle, cycle_member);
        E.set(kFirstCycle, [&](int k) { return cycle_member(k) && runs[k].gm.first; });
        E.put_flags();
        E.phase(kPhaseCycleStart, [&] { batch_precondition(E, -1); });
        // step 0 for every member in the cycle, then look ahead one step
        std::vector<std::vector<char>> took(m, std::vector<char>(nm, 0));
        for (int k = 0; k < nm; ++k) took[0][k] = cycle_member(k);
        E.set(kFirstCycle, [](int) { return false; });
        E.put_flags();
        E.phase(kPhaseArnoldi, [&] { batch_arnoldi(E, 0, dcols, hcols, LDH); });
        std::vector<hipEvent_t> done(m, nullptr);
        auto record = [&](int j) {
            if (!done[j]) HIPCHECK(hipEventCreateWithFlags(&done[j], hipEventDisableTiming));
            HIPCHECK(hipEventRecord(done[j], E.s));
        };
        record(0);
        (void)colstride;
        try {
            for (int j = 0;; ++j) {
                if (j + 1 < m) {
                    bool any = false;
                    for (int k = 0; k < nm; ++k) {
                        const GmState &G = runs[k].gm;
                        const int max_it = E.mem[k]->opt.max_lin;
                        took[j + 1][k] = cycle_member(k) && !G.stopped && G.total + j + 1 < max_it;
                        any = any || took[j + 1][k];
                    }
                    if (any) {
                        E.set(kOnCycle, [&](int k) { return took[j + 1][k] != 0; });
                        E.put_flags();
                        E.phase(kPhaseArnoldi + j + 1, [&] {
                            batch_arnoldi(E, j + 1, dcols + (size_t)(j + 1) * colstride,
                                          hcols + (size_t)(j + 1) * colstride, LDH);
                        });
                        record(j + 1);
                    }
                }
                HIPCHECK(hipEventSynchronize(done[j]));
                bool all_stopped = true;
                for (int k = 0; k < nm; ++k) {
                    GmState &G = runs[k].gm;
                    if (!cycle_member(k)) continue;
                    if (G.stopped || !took[j][k]) {
                        G.stopped = true;
                        continue;
                    }
                    const int max_it = E.mem[k]->opt.max_lin;
                    const double *h = hcols + (size_t)j * colstride + (size_t)k * LDH;
                    std::vector<double> &Hh = G.Hh;
                    for (int i = 0; i <= j + 1; ++i) Hh[(size_t)i * m + j] = h[i];
                    for (int i = 0; i < j; ++i) {
                        const double a = Hh[(size_t)i * m + j], bq = Hh[(size_t)(i + 1) * m + j];
                        Hh[(size_t)i * m + j] = G.cs[i] * a + G.sn[i] * bq;
                        Hh[(size_t)(i + 1) * m + j] = -G.sn[i] * a + G.cs[i] * bq;
                    }
                    const double a = Hh[(size_t)j * m + j], bq = Hh[(size_t)(j + 1) * m + j];
                    const double den = std::hypot(a, bq);
                    G.cs[j] = den > 0 ? a / den : 1.0;
                    G.sn[j] = den > 0 ? bq / den : 0.0;
                    Hh[(size_t)j * m + j] = den;
                    Hh[(size_t)(j + 1) * m + j] = 0.0;
                    G.g[j + 1] = -G.sn[j] * G.g[j];
                    G.g[j] = G.cs[j] * G.g[j];
                    G.k = j + 1;
                    const bool breakdown = !(h[j + 1] > 0.0) || !std::isfinite(h[j + 1]);
                    if (std::fabs(G.g[j + 1]) <= G.stop || G.k == m || G.total + G.k >= max_it ||
                        breakdown || !std::isfinite(G.g[j + 1]))
                        G.stopped = true;
                    else
                        all_stopped = false;
                }
                if (all_stopped) break;
            }
        } catch (...) {
            for (hipEvent_t e : done)
                if (e) (void)hipEventDestroy(e);
            throw;
        }
        HIPCHECK(hipStreamSynchronize(E.s));
        for (hipEvent_t e : done)
            if (e) (void)hipEventDestroy(e);
        // the cycle's end: x += Z y, then the true residual
        for (int k = 0; k < nm; ++k) {
            GmState &G = runs[k].gm;
            E.h_k[k] = 0;
            if (!cycle_member(k)) continue;
            const int kk = G.k;
            G.total += kk;
            for (int i = kk - 1; i >= 0; --i) {
                double sacc = G.g[i];
                for (int jj = i + 1; jj < kk; ++jj) sacc -= G.Hh[(size_t)i * m + jj] * G.y[jj];
                G.y[i] = sacc / G.Hh[(size_t)i * m + i];
            }
            for (int i = 0; i < kk; ++i) E.h_ypack[(size_t)k * E.ld_y + i] = G.y[i];
            E.h_k[k] = kk;
        }
        HIPCHECK(hipMemcpyAsync(E.d_ypack, E.h_ypack, (size_t)nm * E.ld_y * sizeof(double),
                                hipMemcpyHostToDevice, E.s));
        HIPCHECK(hipMemcpyAsync(E.d_k, E.h_k, nm * sizeof(int), hipMemcpyHostToDevice, E.s));
        E.set(kOnFinish, cycle_member);
        E.set(kOnCycle, [](int) { return false; });
        E.put_flags();
        E.phase(kPhaseFinish, [&] {
            launchb_axpy(E.s, E.d_mem, E.batch(E.vec, kOnFinish), E.vec.total, E.d_k, E.d_ypack,
                         E.ld_y);
            launchb_spmv(E.s, E.nb, E.d_mem, E.batch(E.spmv, kOnFinish), E.spmv.total, -1);
            launchb_residual(E.s, E.d_mem, E.batch(E.vec, kOnFinish), E.vec.total,
                             E.batch(E.one, kOnFinish), E.one.total, S_RES);
            E.gather(kOnFinish, S_RES, 2);
        });
        E.sync();
        for (int k = 0; k < nm; ++k) {
            GmState &G = runs[k].gm;
            if (!cycle_member(k)) continue;
            const int max_it = E.mem[k]->opt.max_lin;
            G.beta = E.h_scal[(size_t)k * E.ld_scal + 1];
            G.relres = G.beta / G.bnorm;
            G.first = false;
            if (G.relres <= G.rtol) {
                G.status = 0;
                G.in_cycle = false;
            } else if (G.total >= max_it || !std::isfinite(G.relres)) {
                G.status = 1;
                G.in_cycle = false;
            }
        }
        E.set(kOnFinish, [](int) { return false; });
    }
}

}  // namespace

namespace {

// fim_ensemble_run: every member's steps by the state machine of step_impl
// and newton(), in rounds of batched launches
int ensemble_impl(int count, fim_ctx *const *members, int nsteps, const double *dt,
                  fim_step_report *reports, int32_t *status) {
    std::unique_ptr<Ensemble> EP = make_ensemble(count, members);
    Ensemble &E = *EP;
    const int nm = E.nm, m = E.m, LDH = kMaxRestart + 2;
    std::vector<MemRun> runs(nm);
    for (int k = 0; k < nm; ++k) {
        for (int s = 0; s < nsteps; ++s) {
            status[(size_t)k * nsteps + s] = FIM_SKIPPED;
            if (reports) reports[(size_t)k * nsteps + s] = fim_step_report{};
        }
        REQUIRE(dt[(size_t)k * nsteps] > 0, "member %d: dt must be > 0", k);
    }
    // the Hessenberg columns of every step of a cycle, packed by member
    const size_t ncol = (size_t)(m + 1) * nm * LDH;
    double *dcols = E.dalloc<double>(ncol);
    double *hcols = nullptr;
    HIPCHECK(hipHostMalloc((void **)&hcols, ncol * sizeof(double), hipHostMallocDefault));
    struct PinGuard {
        double *p;
        ~PinGuard() { if (p) (void)hipHostFree(p); }
    } pin_guard{hcols};
    int result = FIM_OK;
    auto finish_step = [&](int k, int st_code) {
        MemRun &R = runs[k];
        fim_step_report &r = R.rep;
        r.newton_iters = R.ns.newton;
        r.linear_iters = R.ns.linear;
        r.converged = st_code == FIM_OK;
        r.dt_done = st_code == FIM_OK ? R.dt : 0.0;
        for (int i = 0; i < 3; ++i) {
            r.cnv[i] = R.ns.cnv[i];
            r.mb[i] = R.ns.mb[i];
        }
        r.last_dp = R.ns.last_dp;
        r.last_ds = R.ns.last_ds;
        r.well_res = R.ns.well_res;
        status[(size_t)k * nsteps + R.st] = st_code;
        if (reports) reports[(size_t)k * nsteps + R.st] = r;
        if (st_code != FIM_OK) {
            R.stopped = true;
            result = FIM_NOT_CONVERGED;
            return;
        }
        R.st++;
        R.start_step = true;
        if (R.st >= nsteps) R.stopped = true;
    };
    for (int k = 0; k < nm; ++k) runs[k].stopped = nsteps == 0;
    for (;;) {
        // new steps and sub-steps: the state copies of step_impl
        bool work = false;
        for (int k = 0; k < nm; ++k) {
            MemRun &R = runs[k];
            E.flags[k] &= ~(kSave0 | kSave1);
            if (R.stopped) continue;
            work = true;
            if (R.start_step) {
                R.dt = dt[(size_t)k * nsteps + R.st];
                REQUIRE(R.dt > 0 && std::isfinite(R.dt), "member %d: dt must be > 0", k);
                R.remaining = R.dt;
                R.h = R.dt;
                R.rep = fim_step_report{};
                R.ns = NewtonStats{};
                E.flags[k] |= kSave0;
                R.start_step = false;
                R.start_sub = true;
            }
            if (R.start_sub) {
                R.tdt = std::min(R.h, R.remaining);
                R.it = 0;
                R.last_dp = R.last_ds = INFINITY;
                R.last_viol = 0.0;
                R.forcing = Forcing{};
                E.flags[k] |= kSave1;
                R.start_sub = false;
            }
        }
        if (!work) break;
        if (E.any(kSave0) || E.any(kSave1)) {
            E.put_flags();
            if (E.any(kSave0))
                E.phase(kPhaseSave0, [&] {
                    launchb_state_copy(E.s, E.d_mem, E.statecopy.d, E.d_flags, nm,
                                       E.statecopy.total, E.d_slots, 0, kSave0, 0);
                });
            if (E.any(kSave1))
                E.phase(kPhaseSave1, [&] {
                    launchb_state_copy(E.s, E.d_mem, E.statecopy.d, E.d_flags, nm,
                                       E.statecopy.total, E.d_slots, 1, kSave1, 0);
                });
        }
        // assembly round: properties (step-start accumulation at it = 0),
        // residual and Jacobian, convergence measures
        for (int k = 0; k < nm; ++k) {
            const MemRun &R = runs[k];
            E.h_dt[k] = R.tdt;
            const bool on = !R.stopped;
            E.flags[k] = (E.flags[k] & ~(kOnNewton | kAold | kOnSolve | kOnUpdate | kSave0 | kSave1)) |
                         (on ? kOnNewton : 0) | (on && R.it == 0 ? kAold : 0);
        }
        HIPCHECK(hipMemcpyAsync(E.d_dt, E.h_dt, nm * sizeof(double), hipMemcpyHostToDevice, E.s));
        E.put_flags();
        E.phase(kPhaseAssemble, [&] {
            launchb_props(E.s, E.nb, E.d_mem, E.batch(E.cells, kOnNewton), E.cells.total);
            launchb_assemble(E.s, E.nb, E.d_mem, E.batch(E.cells, kOnNewton), E.cells.total,
                             E.batch(E.wells, kOnNewton), E.wells.total, E.d_dt);
            launchb_conv(E.s, E.nb, E.d_mem, E.batch(E.conv, kOnNewton), E.conv.total,
                         E.batch(E.one, kOnNewton), E.one.total, E.d_dt, S_CONV);
            E.gather(kOnNewton, S_CONV, S_NORM - S_CONV);
        });
        E.sync();
        // the convergence check of newton() for every member
        std::vector<int> fail(nm, 0), ok(nm, 0);
        for (int k = 0; k < nm; ++k) {
            MemRun &R = runs[k];
            R.solve = false;
            if (R.stopped) continue;
            fim_ctx *c = E.mem[k];
            const fim_options &o = c->opt;
            const int nb = c->nb;
            const double *sc = E.h_scal + (size_t)k * E.ld_scal + S_CONV;
            if (R.it > 0) {
                R.last_dp = sc[S_UPD - S_CONV];
                R.last_ds = sc[S_UPD - S_CONV + 1];
                R.last_viol = sc[S_UPD - S_CONV + 2];
            }
            bool finite = std::isfinite(R.last_dp) || R.it == 0;
            bool conv = R.it > 0;
            for (int i = 0; i < nb; ++i) {
                R.ns.cnv[i] = sc[i];
                R.ns.mb[i] = R.tdt * std::fabs(sc[nb + i]) / sc[2 * nb + i];
                finite = finite && std::isfinite(R.ns.cnv[i]) && std::isfinite(R.ns.mb[i]);
                conv = conv && R.ns.cnv[i] <= o.tol_cnv && R.ns.mb[i] <= o.tol_mb;
            }
            const double wmax = sc[3 * nb];
            R.ns.last_dp = R.last_dp;
            R.ns.last_ds = R.last_ds;
            R.ns.well_res = wmax;
            finite = finite && std::isfinite(wmax);
            if (!finite) {
                fail[k] = 1;
                continue;
            }
            conv = conv && wmax <= o.tol_well && R.last_dp <= o.tol_dp && R.last_ds <= o.tol_ds;
            if (conv) {
                if (R.last_viol <= kSatSlack) ok[k] = 1;
                else fail[k] = 1;
                continue;
            }
            if (R.it >= o.max_newton) {
                fail[k] = 1;
                continue;
            }
            R.solve = true;
        }
        // solve and update for the members that go on
        bool anysolve = false;
        for (int k = 0; k < nm; ++k) anysolve = anysolve || runs[k].solve;
        if (anysolve) {
            E.set(kOnSolve, [&](int k) { return runs[k].solve; });
            E.put_flags();
            E.phase(kPhaseSetup, [&] { batch_prec_setup(E); });
            batch_gmres(E, runs, dcols, hcols);
            for (int k = 0; k < nm; ++k) {
                MemRun &R = runs[k];
                if (!R.solve) continue;
                const GmState &G = R.gm;
                R.ns.linear += G.total;
                R.ns.newton += 1;
                if (G.status != 0 && !(std::isfinite(G.relres) && G.relres < 1.0)) {
                    fail[k] = 1;
                    R.solve = false;
                }
            }
            E.set(kOnUpdate, [&](int k) { return runs[k].solve; });
            E.set(kOnSolve, [](int) { return false; });
            E.put_flags();
            E.phase(kPhaseUpdate, [&] {
                launchb_newton_update(E.s, E.nb, E.d_mem, E.batch(E.conv, kOnUpdate),
                                      E.conv.total, E.batch(E.one, kOnUpdate), E.one.total, S_UPD);
            });
            for (int k = 0; k < nm; ++k)
                if (runs[k].solve) runs[k].it++;
        }
        // accepted and failed sub-steps (step_impl)
        for (int k = 0; k < nm; ++k) {
            MemRun &R = runs[k];
            E.flags[k] &= ~(kRestore0 | kRestore1 | kOnUpdate);
            if (ok[k]) {
                R.remaining -= R.tdt;
                if (R.rep.nsub < FIM_MAX_SUB) R.rep.dt_sub[R.rep.nsub] = R.tdt;
                R.rep.nsub++;
                R.start_sub = true;
                if (!(R.remaining > 1e-12 * R.dt)) finish_step(k, FIM_OK);
            } else if (fail[k]) {
                E.flags[k] |= kRestore1;
                R.rep.cuts++;
                if (R.rep.cuts > E.mem[k]->opt.max_cuts) {
                    E.flags[k] |= kRestore0;
                    finish_step(k, FIM_NOT_CONVERGED);
                } else {
                    R.h = 0.5 * R.tdt;
                    R.start_sub = true;
                }
            }
        }
        if (E.any(kRestore1) || E.any(kRestore0)) {
            E.put_flags();
            if (E.any(kRestore1))
                E.phase(kPhaseRestore1, [&] {
                    launchb_state_copy(E.s, E.d_mem, E.statecopy.d, E.d_flags, nm,
                                       E.statecopy.total, E.d_slots, 1, 0, kRestore1);
                });
            if (E.any(kRestore0))
                E.phase(kPhaseRestore0, [&] {
                    launchb_state_copy(E.s, E.d_mem, E.statecopy.d, E.d_flags, nm,
                                       E.statecopy.total, E.d_slots, 0, 0, kRestore0);
                });
        }
    }
    HIPCHECK(hipStreamSynchronize(E.s));
    // the step-start accumulation of every member's next step, on its stream
    for (fim_ctx *c : E.mem) {
        props(c, true);
        c->jac_ready = false;
        c->prec_ready = false;
    }
    for (fim_ctx *c : E.mem) c->sync();
    return result;
}

}  // namespace

// ---------------------------------------------------------------------------
// autotuner of the ensemble's block-Jacobi ILU(0) boxes
//
// The box sets both the ILU(0) preconditioner (fewer, larger boxes: fewer
// linear iterations) and the cost of one application (longer hyperplane
// sweeps per workgroup, fewer workgroups).  The tuner times trial steps of
// the whole batched ensemble from its current state with every candidate
// box, keeps the fastest, and caches the choice per (block size, size
// bucket of the median member, device); a later call with the same key
// applies the cached box without trials.  Candidates keep 64 pencils per
// box (the batched ILU(0) launches take one workgroup size).

namespace {

const int kTuneBoxes[][3] = {{8, 8, 8}, {8, 8, 16}, {8, 8, 4}, {16, 4, 8}, {4, 16, 8}, {16, 4, 16}};
constexpr int kTuneCand = sizeof(kTuneBoxes) / sizeof(kTuneBoxes[0]);

struct SavedState {
    double *P = nullptr, *Sw = nullptr, *X = nullptr, *pbhp = nullptr;
    int8_t *flag = nullptr;
};

std::string tune_key(const std::vector<fim_ctx *> &mem) {
    std::vector<int> n;
    for (const fim_ctx *c : mem) n.push_back(c->n);
    std::sort(n.begin(), n.end());
    const int med = n[n.size() / 2];
    int bucket = 0;
    while ((1 << (bucket + 1)) <= med) ++bucket;            // floor(log2(median cells))
    hipDeviceProp_t prop{};
    HIPCHECK(hipGetDeviceProperties(&prop, mem[0]->dev));
    std::string name = prop.gcnArchName;
    for (char &ch : name)
        if (ch == ' ') ch = '_';
    char buf[256];
    std::snprintf(buf, sizeof buf, "nb%d_cells2^%d_%s", mem[0]->nb, bucket, name.c_str());
    return buf;
}

bool tune_lookup(const char *path, const std::string &key, int (&box)[3]) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char k[256];
    int t[3];
    bool found = false;
    while (std::fscanf(f, "%255s %d %d %d", k, &t[0], &t[1], &t[2]) == 4)
        if (key == k) {
            for (int a = 0; a < 3; ++a) box[a] = t[a];
            found = true;                                   // the last entry wins
        }
    std::fclose(f);
    return found;
}

void set_box(fim_ctx *c, const int (&box)[3]) {
    fim_options o = c->opt;
    o.tile_nx = box[0];
    o.tile_ny = box[1];
    o.tile_nz = box[2];
    REQUIRE(fim_set_options(c, &o) == FIM_OK, "%s", g_err.c_str());
}

int tune_impl(int count, fim_ctx *const *members, double dt, int trial_steps, const char *cache,
              fim_tune_report *rep) {
    REQUIRE(count >= 1 && members, "members are required");
    REQUIRE(dt > 0 && std::isfinite(dt), "dt must be > 0");
    REQUIRE(trial_steps >= 1, "trial_steps must be >= 1");
    std::vector<fim_ctx *> mem(members, members + count);
    for (int k = 0; k < count; ++k) {
        REQUIRE(members[k], "member %d is NULL", k);
        if (!members[k]->state_set) {
            set_err("member %d: state not set", k);
            throw StateError();
        }
    }
    fim_tune_report r{};
    r.ncand = kTuneCand;
    for (int c = 0; c < kTuneCand; ++c)
        for (int a = 0; a < 3; ++a) r.cand[c][a] = kTuneBoxes[c][a];
    const std::string key = tune_key(mem);
    int best[3];
    if (tune_lookup(cache, key, best)) {
        for (fim_ctx *c : mem) set_box(c, best);
        r.from_cache = 1;
        for (int a = 0; a < 3; ++a) r.box[a] = best[a];
        if (rep) *rep = r;
        return FIM_OK;
    }
    // the members' states, to start every trial from and to leave them in
    std::vector<SavedState> saved(count);
    std::vector<void *> bufs;
    struct Free {
        std::vector<void *> &b;
        ~Free() {
            for (void *p : b) (void)hipFree(p);
        }
    } free_bufs{bufs};
    auto dal = [&](size_t bytes) {
        void *p = nullptr;
        HIPCHECK(hipMalloc(&p, std::max<size_t>(bytes, 8)));
        bufs.push_back(p);
        return p;
    };
    auto copy = [&](fim_ctx *c, SavedState &S, bool save) {
        const size_t n = c->n;
        auto cp = [&](void *a, void *b, size_t bytes) {
            HIPCHECK(hipMemcpyAsync(save ? a : b, save ? b : a, bytes, hipMemcpyDeviceToDevice, c->s));
        };
        cp(S.P, c->P, n * 8);
        cp(S.Sw, c->Sw, n * 8);
        cp(S.X, c->X, n * 8);
        cp(S.flag, c->flag, n);
        if (c->nw) cp(S.pbhp, c->pbhp, c->nw * 8);
        if (!save) props(c, true);
    };
    for (int k = 0; k < count; ++k) {
        fim_ctx *c = mem[k];
        SavedState &S = saved[k];
        S.P = (double *)dal((size_t)c->n * 8);
        S.Sw = (double *)dal((size_t)c->n * 8);
        S.X = (double *)dal((size_t)c->n * 8);
        S.flag = (int8_t *)dal(c->n);
        S.pbhp = (double *)dal((size_t)std::max(c->nw, 1) * 8);
        copy(c, S, true);
    }
    for (fim_ctx *c : mem) c->sync();
    const int orig[3] = {mem[0]->opt.tile_nx, mem[0]->opt.tile_ny, mem[0]->opt.tile_nz};
    std::vector<double> dts((size_t)count * trial_steps, dt);
    std::vector<int32_t> st((size_t)count * trial_steps);
    double best_ms = INFINITY;
    int bi = -1;
    for (int cand = 0; cand < kTuneCand; ++cand) {
        for (fim_ctx *c : mem) set_box(c, kTuneBoxes[cand]);
        for (int k = 0; k < count; ++k) copy(mem[k], saved[k], false);
        for (fim_ctx *c : mem) c->sync();
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = ensemble_impl(count, members, trial_steps, dts.data(), nullptr, st.data());
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        r.trial_ms[cand] = rc == FIM_OK ? ms : INFINITY;
        r.trials++;
        if (rc == FIM_OK && ms < best_ms) {
            best_ms = ms;
            bi = cand;
        }
    }
    if (bi < 0) {
        // no candidate finished its trial steps: leave the members as they were
        for (fim_ctx *c : mem) {
            const int o[3] = {orig[0], orig[1], orig[2]};
            set_box(c, o);
        }
        for (int k = 0; k < count; ++k) copy(mem[k], saved[k], false);
        for (fim_ctx *c : mem) c->sync();
        set_err("no candidate box finished the trial steps");
        if (rep) *rep = r;
        return FIM_NOT_CONVERGED;
    }
    for (int a = 0; a < 3; ++a) best[a] = kTuneBoxes[bi][a];
    for (fim_ctx *c : mem) set_box(c, best);
    for (int k = 0; k < count; ++k) copy(mem[k], saved[k], false);
    for (fim_ctx *c : mem) c->sync();
    if (cache) {
        FILE *f = std::fopen(cache, "a");
        REQUIRE(f, "cannot open the tuning cache %s", cache);
        std::fprintf(f, "%s %d %d %d\n", key.c_str(), best[0], best[1], best[2]);
        std::fclose(f);
    }
    for (int a = 0; a < 3; ++a) r.box[a] = best[a];
    if (rep) *rep = r;
    return FIM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// permeability (the ROCK input of Sec. 3.2.3): new kx, ky, kz, then the
// static precompute that depends on them again (transmissibilities and the
// Peaceman well indices; explicit well indices stay)

static int set_perm_impl(fim_ctx *c, const double *kx, const double *ky, const double *kz,
                         bool dev) {
    const size_t b = (size_t)c->n * 8;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHECK(hipMemcpyAsync(c->kx, kx, b, kind, c->s));
    HIPCHECK(hipMemcpyAsync(c->ky, ky, b, kind, c->s));
    HIPCHECK(hipMemcpyAsync(c->kz, kz, b, kind, c->s));
    if (c->nperf)
        HIPCHECK(hipMemcpyAsync(c->wi, c->wi_explicit.data(), (size_t)c->nperf * 8,
                                hipMemcpyHostToDevice, c->s));
    launch_static(c->s, c->g, c->dx, c->dy, c->dz, c->top, c->kx, c->ky, c->kz, c->poro, c->vol,
                  c->depth, c->pvref, c->tx, c->ty, c->tz);
    launch_peaceman(c->s, c->g, c->nperf, c->pcell, c->pwell, c->dx, c->dy, c->dz, c->kx, c->ky,
                    c->wrw, c->wskin, c->wi);
    HIPCHECK(hipGetLastError());
    c->sync();                 // the explicit indices are read from host memory
    c->jac_ready = false;
    c->prec_ready = false;
    return FIM_OK;
}

// ---------------------------------------------------------------------------
// state transfer

static void put_state(fim_ctx *c, const double *p, const double *sw, const double *x3,
                      const int8_t *flag, const double *bhp, bool dev, bool reset_start) {
    REQUIRE(p && sw, "p and sw are required");
    const size_t n = c->n;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHECK(hipMemcpyAsync(c->P, p, n * 8, kind, c->s));
    HIPCHECK(hipMemcpyAsync(c->Sw, sw, n * 8, kind, c->s));
    if (x3 && c->nb == 3) HIPCHECK(hipMemcpyAsync(c->X, x3, n * 8, kind, c->s));
    else launch_scale_copy(c->s, (long)n, nullptr, 0.0, c->X);
    if (flag && c->nb == 3) HIPCHECK(hipMemcpyAsync(c->flag, flag, n, kind, c->s));
    else HIPCHECK(hipMemsetAsync(c->flag, 0, n, c->s));
    std::vector<double> pb(c->nw);
    if (bhp) {
        for (int wl = 0; wl < c->nw; ++wl) pb[wl] = bhp[wl];
    } else if (c->nw) {
        // BHP wells start at their target, rate wells at the mean pressure of
        // their perforated cells
        std::vector<double> ph(n);
        if (dev) {
            HIPCHECK(hipMemcpyAsync(ph.data(), p, n * 8, hipMemcpyDeviceToHost, c->s));
            c->sync();
        } else {
            std::memcpy(ph.data(), p, n * 8);
        }
        std::vector<int> cells(c->nperf);
        HIPCHECK(hipMemcpy(cells.data(), c->pcell, c->nperf * sizeof(int), hipMemcpyDeviceToHost));
        for (int wl = 0; wl < c->nw; ++wl) {
            if (c->wctrl[wl] == FIM_BHP) {
                pb[wl] = c->wtarget[wl];
            } else {
                double sacc = 0;
                for (int q = c->wps[wl]; q < c->wps[wl + 1]; ++q) sacc += ph[cells[q]];
                pb[wl] = sacc / (c->wps[wl + 1] - c->wps[wl]);
            }
        }
    }
    if (c->nw) {
        HIPCHECK(hipMemcpyAsync(c->pbhp, pb.data(), c->nw * 8, hipMemcpyHostToDevice, c->s));
    }
    if (reset_start) props(c, true);
    c->sync();
    c->state_set = true;
    c->jac_ready = false;
}

// ---------------------------------------------------------------------------
// the step without device allocation (fim_step_noalloc)
//
// The reduction partials and the scalar slots of a step live in one static
// device array, `scratch`: every GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address); the device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and is kept per device.

constexpr size_t kNoAllocPartials = (size_t)32 * 2048;   // reduction partials
constexpr size_t kNoAllocDoubles = kNoAllocPartials + S_COUNT;   // + scalar slots
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};

// the device address of `scratch` on device dev
static double *scratch_on(int dev) {
    REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        HIPCHECK(hipGetDevice(&cur));
        if (cur != dev) HIPCHECK(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHECK(hipSetDevice(cur));
        HIPCHECK(e);
        REQUIRE(ptr, "no device address for the static scratch array on device %d", dev);
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_dev[dev];
}

// doubles of reduction partials one step of the context writes: the
// Gram-Schmidt products (up to restart + 1 per column block), the
// convergence measures and the Newton update
static size_t step_partials(const fim_ctx *c) {
    const size_t vb = (size_t)vec_blocks(c->nvec);
    const size_t cb = (size_t)conv_blocks(c->n), ub = (size_t)update_blocks(c->n);
    return std::max({(size_t)(c->m + 1) * vb, (size_t)(3 * c->nb + 1) * cb, 3 * ub, vb});
}

// fim_step with the context's partials and scalar slots replaced by the
// static array, eager launches (no graph executable is instantiated) and no
// profiling events; everything else is the context's, allocated at create
static int step_noalloc_impl(fim_ctx *c, double dt, fim_step_report *rep) {
    const size_t need = step_partials(c);
    REQUIRE(need <= kNoAllocPartials,
            "fim_step_noalloc: the step needs %zu doubles of reduction scratch, the static "
            "array holds %zu (restart %d on %ld vector entries; restart <= 31 always fits)",
            need, kNoAllocPartials, c->m, c->nvec);
    double *base = scratch_on(c->dev);
    struct Swap {
        fim_ctx *c;
        double *partials, *scal;
        int graphs, profile;
        ~Swap() {
            c->partials = partials;
            c->scal = scal;
            c->opt.graphs = graphs;
            c->opt.profile = profile;
        }
    } keep{c, c->partials, c->scal, c->opt.graphs, c->opt.profile};
    c->partials = base;
    c->scal = base + kNoAllocPartials;
    c->opt.graphs = 0;
    c->opt.profile = 0;
    // the scalar slots keep the last call's values (perhaps another
    // context's): clear them with a kernel (no memset node)
    launch_scale_copy(c->s, S_COUNT, nullptr, 0.0, c->scal);
    return step_impl(c, dt, rep);
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *fim_last_error(void) { return g_err.c_str(); }

int fim_create(const fim_grid *grid, const fim_rock *rock, const fim_fluid *fluid,
               int32_t nwells, const fim_well *wells, const fim_options *opt, void *hip_stream,
               fim_ctx **out) {
    return guarded([&] { return create_impl(grid, rock, fluid, nwells, wells, opt, hip_stream, out); });
}

void fim_destroy(fim_ctx *ctx) { delete ctx; }

int fim_sizes(const fim_ctx *c, int32_t *ncells, int32_t *nb, int32_t *nwells, int32_t *nnzb,
              int32_t *nprops) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        if (ncells) *ncells = c->n;
        if (nb) *nb = c->nb;
        if (nwells) *nwells = c->nw;
        if (nnzb) *nnzb = c->nnzb;
        if (nprops) *nprops = (c->nb == 2) ? Rec<2>::N : Rec<3>::N;
        return FIM_OK;
    });
}

int fim_set_options(fim_ctx *c, const fim_options *opt) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        check_options(opt);
        REQUIRE(opt->amg_exact == c->opt.amg_exact,
                "amg_exact is fixed when the context is created (%d, not %d)", c->opt.amg_exact,
                opt->amg_exact);
        REQUIRE(opt->amg_exact_mode == c->opt.amg_exact_mode,
                "amg_exact_mode is fixed when the context is created (%d, not %d)",
                c->opt.amg_exact_mode, opt->amg_exact_mode);
        c->sync();
        c->drop_graphs();        // captured steps depend on the options and buffers
        if (opt->restart > c->m) {
            c->sync();
            alloc_krylov(c, opt->restart);
        } else {
            c->m = opt->restart;
        }
        c->opt = *opt;
        build_subcycle(c);
        build_ilu(c);
        ensure_mixed(c);
        c->prec_ready = false;
        return FIM_OK;
    });
}

int fim_set_state(fim_ctx *c, const double *p, const double *sw, const double *x3,
                  const int8_t *flag, const double *bhp) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        put_state(c, p, sw, x3, flag, bhp, false, true);
        return FIM_OK;
    });
}

int fim_set_state_dev(fim_ctx *c, const double *p, const double *sw, const double *x3,
                      const int8_t *flag, const double *bhp) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        HIPCHECK(hipEventRecord(c->ev_user, c->user_s));
        HIPCHECK(hipStreamWaitEvent(c->s, c->ev_user, 0));
        put_state(c, p, sw, x3, flag, bhp, true, true);
        return FIM_OK;
    });
}

int fim_set_iterate(fim_ctx *c, const double *p, const double *sw, const double *x3,
                    const int8_t *flag, const double *bhp) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        if (!c->state_set) {
            set_err("state not set (call fim_set_state first)");
            throw StateError();
        }
        put_state(c, p, sw, x3, flag, bhp, false, false);
        return FIM_OK;
    });
}

int fim_get_state(fim_ctx *c, double *p, double *sw, double *x3, int8_t *flag, double *bhp) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        const size_t n = c->n;
        if (p) HIPCHECK(hipMemcpyAsync(p, c->P, n * 8, hipMemcpyDeviceToHost, c->s));
        if (sw) HIPCHECK(hipMemcpyAsync(sw, c->Sw, n * 8, hipMemcpyDeviceToHost, c->s));
        if (x3) HIPCHECK(hipMemcpyAsync(x3, c->X, n * 8, hipMemcpyDeviceToHost, c->s));
        if (flag) HIPCHECK(hipMemcpyAsync(flag, c->flag, n, hipMemcpyDeviceToHost, c->s));
        if (bhp && c->nw)
            HIPCHECK(hipMemcpyAsync(bhp, c->pbhp, c->nw * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        return FIM_OK;
    });
}

int fim_step(fim_ctx *c, double dt_days, fim_step_report *rep) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        return step_impl(c, dt_days, rep);
    });
}

int fim_step_noalloc(fim_ctx *c, double dt_days, fim_step_report *rep) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        return step_noalloc_impl(c, dt_days, rep);
    });
}

int fim_adjoint_gradient(fim_ctx *c, int32_t nsteps, const double *dt, const double *q_obs,
                         int32_t checkpoint_every, double *grad, fim_adjoint_report *rep) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        return adjoint_impl(c, nsteps, dt, q_obs, checkpoint_every, grad, rep);
    });
}

int fim_set_perm(fim_ctx *c, const double *kx, const double *ky, const double *kz) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        REQUIRE(kx && ky && kz, "kx, ky and kz are required");
        for (int q = 0; q < c->n; ++q)
            REQUIRE(kx[q] >= 0 && ky[q] >= 0 && kz[q] >= 0, "permeability must be >= 0 (cell %d)", q);
        return set_perm_impl(c, kx, ky, kz, false);
    });
}

int fim_set_perm_dev(fim_ctx *c, const double *kx, const double *ky, const double *kz) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        REQUIRE(kx && ky && kz, "kx, ky and kz are required");
        HIPCHECK(hipEventRecord(c->ev_user, c->user_s));
        HIPCHECK(hipStreamWaitEvent(c->s, c->ev_user, 0));
        return set_perm_impl(c, kx, ky, kz, true);
    });
}

int fim_ensemble_run(int32_t count, fim_ctx *const *members, int32_t nsteps, const double *dt,
                     fim_step_report *reports, int32_t *status) {
    return guarded([&]() -> int {
        REQUIRE(count >= 0 && nsteps >= 0, "count and nsteps must be >= 0");
        if (count == 0 || nsteps == 0) return FIM_OK;
        REQUIRE(members && dt && status, "members, dt and status are required");
        std::vector<fim_ctx *> seen(members, members + count);
        for (int k = 0; k < count; ++k) REQUIRE(members[k], "member %d is NULL", k);
        std::sort(seen.begin(), seen.end());
        REQUIRE(std::adjacent_find(seen.begin(), seen.end()) == seen.end(),
                "a context appears twice among the members");
        return ensemble_impl(count, members, nsteps, dt, reports, status);
    });
}

int fim_ensemble_tune(int32_t count, fim_ctx *const *members, double dt_days,
                      int32_t trial_steps, const char *cache_path, fim_tune_report *rep) {
    return guarded([&] {
        return tune_impl(count, members, dt_days, trial_steps, cache_path, rep);
    });
}

int fim_get_well_rates(fim_ctx *c, double *q_surf, double *bhp) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        if (!c->state_set) {
            set_err("state not set");
            throw StateError();
        }
        if (c->nw == 0) return FIM_OK;
        props(c, false);
        double *dq = c->partials;   // scratch, >= 3 * nwells doubles
        launch_well_rates(c->s, c->nb, c->wells(), c->P, c->pbhp, c->rec, c->n, dq);
        if (q_surf) HIPCHECK(hipMemcpyAsync(q_surf, dq, c->nw * 3 * 8, hipMemcpyDeviceToHost, c->s));
        if (bhp) HIPCHECK(hipMemcpyAsync(bhp, c->pbhp, c->nw * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        return FIM_OK;
    });
}

int fim_static(fim_ctx *c, double *vol, double *depth, double *pvref, double *tx, double *ty,
               double *tz, double *wi_out) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        const size_t b = (size_t)c->n * 8;
        if (vol) HIPCHECK(hipMemcpyAsync(vol, c->vol, b, hipMemcpyDeviceToHost, c->s));
        if (depth) HIPCHECK(hipMemcpyAsync(depth, c->depth, b, hipMemcpyDeviceToHost, c->s));
        if (pvref) HIPCHECK(hipMemcpyAsync(pvref, c->pvref, b, hipMemcpyDeviceToHost, c->s));
        if (tx) HIPCHECK(hipMemcpyAsync(tx, c->tx, b, hipMemcpyDeviceToHost, c->s));
        if (ty) HIPCHECK(hipMemcpyAsync(ty, c->ty, b, hipMemcpyDeviceToHost, c->s));
        if (tz) HIPCHECK(hipMemcpyAsync(tz, c->tz, b, hipMemcpyDeviceToHost, c->s));
        std::vector<double> ws(c->nperf);
        if (wi_out && c->nperf)
            HIPCHECK(hipMemcpyAsync(ws.data(), c->wi, c->nperf * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        if (wi_out)
            for (int q = 0; q < c->nperf; ++q) wi_out[c->perf_src[q]] = ws[q];
        return FIM_OK;
    });
}

int fim_props(fim_ctx *c, double *out) {
    return guarded([&] {
        REQUIRE(c && out, "context and out are required");
        if (!c->state_set) {
            set_err("state not set");
            throw StateError();
        }
        props(c, false);
        const int N = (c->nb == 2) ? Rec<2>::N : Rec<3>::N;
        HIPCHECK(hipMemcpyAsync(out, c->rec, (size_t)N * c->n * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        return FIM_OK;
    });
}

int fim_assemble(fim_ctx *c, double dt, double *Rout, int32_t *rowptr, int32_t *colind,
                 double *valout) {
    return guarded([&] {
        REQUIRE(c, "context is NULL");
        REQUIRE(dt > 0, "dt must be > 0");
        if (!c->state_set) {
            set_err("state not set");
            throw StateError();
        }
        props(c, false);
        assemble(c, dt);
        HIPCHECK(hipGetLastError());
        if (Rout) HIPCHECK(hipMemcpyAsync(Rout, c->R, c->nvec * 8, hipMemcpyDeviceToHost, c->s));
        if (rowptr)
            HIPCHECK(hipMemcpyAsync(rowptr, c->rowptr, (c->nrows + 1) * 4, hipMemcpyDeviceToHost, c->s));
        if (colind)
            HIPCHECK(hipMemcpyAsync(colind, c->colind, (size_t)c->nnzb * 4, hipMemcpyDeviceToHost, c->s));
        if (valout)
            HIPCHECK(hipMemcpyAsync(valout, c->val, (size_t)c->nnzb * c->nb * c->nb * 8,
                                    hipMemcpyDeviceToHost, c->s));
        c->sync();
        return FIM_OK;
    });
}

int fim_precond_apply(fim_ctx *c, const double *xh, double *yh) {
    return guarded([&] {
        REQUIRE(c && xh && yh, "context, x and y are required");
        if (!c->jac_ready) {
            set_err("no assembled Jacobian (call fim_assemble first)");
            throw StateError();
        }
        prec_setup(c);
        HIPCHECK(hipMemcpyAsync(c->b, xh, c->nvec * 8, hipMemcpyHostToDevice, c->s));
        if (c->mixed) {
            precondition<double, float>(c, c->b, nullptr, c->V32, c->Z32);
            launch_to_double(c->s, c->nvec, c->Z32, c->t);
        } else {
            precondition<double, double>(c, c->b, nullptr, nullptr, c->t);
        }
        HIPCHECK(hipMemcpyAsync(yh, c->t, c->nvec * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        return FIM_OK;
    });
}

int fim_linear_solve(fim_ctx *c, const double *bh, double *xh, int32_t *iters, double *relres) {
    return guarded([&] {
        REQUIRE(c && bh && xh, "context, b and x are required");
        if (!c->jac_ready) {
            set_err("no assembled Jacobian (call fim_assemble first)");
            throw StateError();
        }
        prec_setup(c);
        HIPCHECK(hipMemcpyAsync(c->b, bh, c->nvec * 8, hipMemcpyHostToDevice, c->s));
        int it = 0;
        double rr = 0;
        const int st = gmres(c, c->b, c->x, c->opt.max_lin, c->opt.lin_rtol, false, &it, &rr);
        HIPCHECK(hipMemcpyAsync(xh, c->x, c->nvec * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        if (iters) *iters = it;
        if (relres) *relres = rr;
        return st == 0 ? FIM_OK : FIM_NOT_CONVERGED;
    });
}

int fim_amg_level(fim_ctx *c, int32_t level, int32_t *dims, double *A) {
    return guarded([&] {
        REQUIRE(c && dims, "context and dims are required");
        REQUIRE(uses_cpr(c->opt), "the context's preconditioner has no AMG stage");
        REQUIRE(level >= 0 && level < (int)c->lv.size(), "level %d of %zu", level, c->lv.size());
        if (!c->jac_ready) {
            set_err("no assembled Jacobian (call fim_assemble first)");
            throw StateError();
        }
        if (!c->prec_ready) prec_setup(c);
        const AmgLevel &L = c->lv[level];
        dims[0] = L.nx;
        dims[1] = L.ny;
        dims[2] = L.nz;
        dims[3] = L.nw;
        if (!A) return FIM_OK;
        const int ncs = 2 * L.half, nc = L.nx * L.ny * L.nz, N = nc + L.nw;
        std::vector<double> a((size_t)7 * ncs), aww(std::max(L.nw, 1)), acw(std::max(L.nslot, 1)),
            awc(std::max(L.nslot, 1));
        std::vector<int> cps(ncs + 1), cslot(std::max(L.nslot, 1)), swell(std::max(L.nslot, 1)),
            scell(std::max(L.nslot, 1)), sps(L.nw + 1);
        auto get = [&](void *dst, const void *src, size_t bytes) {
            if (bytes) HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->s));
        };
        get(a.data(), L.a, a.size() * 8);
        get(aww.data(), L.aww, (size_t)L.nw * 8);
        get(acw.data(), L.acw, (size_t)L.nslot * 8);
        get(awc.data(), L.awc, (size_t)L.nslot * 8);
        get(cps.data(), L.cps, cps.size() * 4);
        get(cslot.data(), L.cslot, (size_t)L.nslot * 4);
        get(swell.data(), L.swell, (size_t)L.nslot * 4);
        get(scell.data(), L.scell, (size_t)L.nslot * 4);
        get(sps.data(), L.sps, sps.size() * 4);
        c->sync();
        // split index (colour * half + (c >> 1), c = i + nxp (j + ny k)) <-> natural cell
        std::vector<int> nat_of(ncs, -1);
        auto split = [&](int i, int j, int k) {
            const int cc = i + L.nxp * (j + L.ny * k);
            return (((i + j + k) & 1) ? L.half : 0) + (cc >> 1);
        };
        for (int k = 0; k < L.nz; ++k)
            for (int j = 0; j < L.ny; ++j)
                for (int i = 0; i < L.nx; ++i) nat_of[split(i, j, k)] = i + L.nx * (j + L.ny * k);
        std::fill(A, A + (size_t)N * N, 0.0);
        const int di[7] = {0, -1, 1, 0, 0, 0, 0}, dj[7] = {0, 0, 0, -1, 1, 0, 0},
                  dk[7] = {0, 0, 0, 0, 0, -1, 1};
        for (int k = 0; k < L.nz; ++k)
            for (int j = 0; j < L.ny; ++j)
                for (int i = 0; i < L.nx; ++i) {
                    const int sp = split(i, j, k), row = i + L.nx * (j + L.ny * k);
                    for (int d = 0; d < 7; ++d) {
                        const int ni = i + di[d], nj = j + dj[d], nk = k + dk[d];
                        if (ni < 0 || nj < 0 || nk < 0 || ni >= L.nx || nj >= L.ny || nk >= L.nz)
                            continue;
                        A[(size_t)row * N + ni + L.nx * (nj + L.ny * nk)] += a[(size_t)d * ncs + sp];
                    }
                    for (int q = cps[sp]; q < cps[sp + 1]; ++q)
                        A[(size_t)row * N + nc + swell[cslot[q]]] += acw[cslot[q]];
                }
        for (int w = 0; w < L.nw; ++w) {
            const size_t row = (size_t)(nc + w) * N;
            A[row + nc + w] += aww[w];
            for (int q = sps[w]; q < sps[w + 1]; ++q) A[row + nat_of[scell[q]]] += awc[q];
        }
        return FIM_OK;
    });
}

int fim_amg_coarse_solve(fim_ctx *c, const double *b, double *x) {
    return guarded([&] {
        REQUIRE(c && b && x, "context, b and x are required");
        REQUIRE(uses_cpr(c->opt), "the context's preconditioner has no AMG stage");
        if (!c->jac_ready) {
            set_err("no assembled Jacobian (call fim_assemble first)");
            throw StateError();
        }
        if (!c->prec_ready) prec_setup(c);
        AmgLevel L = c->lv.back();
        const int nc = L.nx * L.ny * L.nz, ncs = 2 * L.half, n = ncs + L.nw;
        // natural order <-> the level's colour-split order (padded entries 0)
        std::vector<double> bs(n, 0.0), xs(n);
        auto split = [&](int cn) {
            const int i = cn % L.nx, j = (cn / L.nx) % L.ny, k = cn / (L.nx * L.ny);
            const int cc = i + L.nxp * (j + L.ny * k);
            return (((i + j + k) & 1) ? L.half : 0) + (cc >> 1);
        };
        for (int cn = 0; cn < nc; ++cn) bs[split(cn)] = b[cn];
        for (int w = 0; w < L.nw; ++w) bs[ncs + w] = b[nc + w];
        // private right-hand side and result: the level's own arrays are left alone
        double *db = c->alloc<double>(n), *dx = c->alloc<double>(n);
        HIPCHECK(hipMemcpyAsync(db, bs.data(), n * 8, hipMemcpyHostToDevice, c->s));
        L.b = db;
        L.x = dx;
        if (c->exact_on) exact_apply(c, L);
        else launch_amg_coarsest_solve(c->s, L, c->Minv);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(xs.data(), dx, n * 8, hipMemcpyDeviceToHost, c->s));
        c->sync();
        c->release(db);
        c->release(dx);
        for (int cn = 0; cn < nc; ++cn) x[cn] = xs[split(cn)];
        for (int w = 0; w < L.nw; ++w) x[nc + w] = xs[ncs + w];
        return FIM_OK;
    });
}

int fim_bsr_spmv(int32_t nrows, int32_t nb, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const double *x, double *y, void *hip_stream) {
    return guarded([&] {
        REQUIRE(nb == 2 || nb == 3, "nb must be 2 or 3");
        REQUIRE(nrows >= 0, "nrows must be >= 0");
        if (nrows == 0) return FIM_OK;
        REQUIRE(rowptr && colind && val && x && y, "device pointers are required");
        launch_spmv(static_cast<hipStream_t>(hip_stream), nb, nrows, rowptr, colind, val, x, y);
        HIPCHECK(hipGetLastError());
        return FIM_OK;
    });
}

}  // extern "C"
