// fim_internal.h - device data layout and kernel launchers of libfim.so.
//
// Layout in HBM (one context):
//   state        P, Sw, X [n] fp64, flag [n] int8, pbhp [nw]  (structure of arrays)
//   static       depth, pvref, tx, ty, tz [n]                 (cell-owned + faces)
//   properties   rec [NREC][n]: the exported property record followed by
//                d(b_j)/dP for each phase (used by injector perforations)
//   system       R [(n+nw)*nb] interleaved; BSR rowptr [n+nw+1], colind [nnzb],
//                val [nnzb][nb][nb] row-major blocks; diagpos [n+nw]
//   Krylov       V [(m+1)][(n+nw)*nb], w, z, x, b, r [(n+nw)*nb]; dinv [n+nw][nb][nb]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fim {

constexpr int kMaxTableRows = 64;
constexpr int kBlock = 256;          // threads per block of the cell/vector kernels
constexpr int kMaxRestart = 40;       // GMRES restart length cap (registers of multidot)

// Workgroups are handed to the eight XCDs round-robin (block b to XCD
// b mod 8), and every XCD has its own L2.  xcd_block maps the hardware block
// index to a logical one so that each XCD walks one contiguous run of
// logical blocks in dispatch order: rows that share vector entries (stencil
// neighbours) are then served by one L2 instead of being fetched into all
// eight.  A bijection on [0, nblk) for any nblk.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nblk) {
    const int q = nblk / kXcds, r = nblk % kXcds;
    const int x = b % kXcds, j = b / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

enum { kProd = 0, kInjWater = 1, kInjGas = 2 };
enum { kBhp = 0, kRate = 1 };
enum { kUnsat = 0, kSat = 1 };

// Index map of the property record for block size NB (NB phases).
template <int NB>
struct Rec {
    static constexpr int G = NB + 1;                   // value + NB derivatives
    static constexpr int LAM = 0;                      // NB groups: kr_j b_j / mu_j
    static constexpr int LAMOG = NB * G;               // NB == 3: Rs * Lam_o
    static constexpr int LT = LAMOG + (NB == 3 ? G : 0);   // total mobility
    static constexpr int GAM = LT + G;                 // NB groups: rho_j / 144
    static constexpr int ACC = GAM + NB * G;           // NB groups: accumulations
    static constexpr int B = ACC + NB * G;             // NB values: 1/B_j
    static constexpr int PV = B + NB;                  // pore volume
    static constexpr int N = PV + 1;                   // exported record length
    static constexpr int DBP = N;                      // NB values: d(1/B_j)/dP
    static constexpr int NREC = N + NB;                // stored record length
};

struct Phys {                       // fluid + rock scalars, passed by value
    int model, nrows;
    double co_us, cmu_us, bw_ref, cw, muw, pw_ref;
    double rho_w, rho_o, rho_g;
    double swc, sor, sgc, nw, no, ng, krw_max, kro_max, krg_max;
    double cr, pref;
    const double *tab;              // device [6][nrows]: p, bo, rs, muo, bg, mug
};

struct Grid {
    int nx, ny, nz, n;
};

struct Wells {                      // perforations sorted by cell within each well
    int nw;
    const int *kind, *ctrl;         // [nw]
    const double *target;           // [nw]
    const int *wps;                 // [nw+1] perforation ranges
    const int *pcell;               // [nperf] perforated cell
    const int *pwell;               // [nperf] owning well
    const double *wi;               // [nperf]
    const int *cps;                 // [n+1] per-cell ranges into cperf
    const int *cperf;               // perforations of each cell, ascending well
};

struct Sys {
    const int *rowptr, *colind, *diagpos;
    double *val, *R;
};

// One level of the pressure AMG hierarchy (structured aggregation).  Cells
// are stored colour-split: split index = colour * half + (c >> 1) with
// c = i + nxp*(j + ny*k) and nxp = nx rounded up to even; wells follow the
// 2*half cell entries in x and b.
struct AmgLevel {
    int nx, ny, nz, nxp, half, nw, nslot;
    unsigned long long mnx, mny, mnxp;   // ceil(2^40 / d) for d = nx, ny, nxp (exact division)
    double *a;              // [7][2*half]: diagonal, -x, +x, -y, +y, -z, +z
    double *aww;            // [nw] well diagonal
    const int *sps;         // [nw+1] well -> slot range
    const int *scell;       // [nslot] split index of the slot's cell
    const int *swell;       // [nslot] well of the slot
    double *acw, *awc;      // [nslot] cell->well and well->cell couplings
    const int *cps;         // [2*half+1] split cell -> range in cslot
    const int *cslot;       // slot ids of each cell
    double *x, *b;          // [2*half + nw]: iterate, right-hand side
    double *xs;             // [nw] the wells' values as the cells of a colour sweep read them
};

// ---- physics kernels (fim_phys.hip) ---------------------------------------
void launch_static(hipStream_t s, Grid g, const double *dx, const double *dy, const double *dz,
                   double top, const double *kx, const double *ky, const double *kz,
                   const double *poro, double *vol, double *depth, double *pvref, double *tx,
                   double *ty, double *tz);
void launch_peaceman(hipStream_t s, Grid g, int nperf, const int *pcell, const int *pwell,
                     const double *dx, const double *dy, const double *dz, const double *kx,
                     const double *ky, const double *rw, const double *skin, double *wi);
void launch_props(hipStream_t s, int nb, Phys f, int n, const double *pvref, const double *P,
                  const double *Sw, const double *X, const int8_t *flag, double *rec,
                  double *aold);
void launch_assemble(hipStream_t s, int nb, Grid g, Phys f, Wells w, Sys sys,
                     const double *depth, const double *tx, const double *ty, const double *tz,
                     const double *P, const double *pbhp, const double *rec, const double *aold,
                     double dt, double *wmeas);
void launch_conv(hipStream_t s, int nb, int n, int nw, const double *rec, const double *R,
                 const double *wmeas, double dt, double *partials, int nparts_blocks,
                 double *out);
void launch_newton_update(hipStream_t s, int nb, Phys f, int n, int nw, const double *y,
                          double ds_max, double dp_max, double *P, double *Sw, double *X,
                          int8_t *flag, double *pbhp, double *partials, int nblocks,
                          double *out);
void launch_well_rates(hipStream_t s, int nb, Wells w, const double *P, const double *pbhp,
                       const double *rec, int n, double *q);
// discrete adjoint (fim_phys.hip, fim_linalg.hip)
void launch_adj_objective(hipStream_t s, int nb, Wells w, int n, const double *P,
                          const double *pbhp, const double *rec, const double *wi_dk,
                          const double *qobs, double *objp, double *objw);
void launch_adj_rhs(hipStream_t s, int nb, Wells w, int n, const double *rec,
                    const double *lam_next, double rdt_next, const double *objp,
                    const double *objw, double *rhs);
void launch_adj_grad(hipStream_t s, int nb, Grid g, Wells w, const double *depth,
                     const double *tx, const double *ty, const double *tz, const double *kx,
                     const double *ky, const double *kz, const double *dx, const double *dy,
                     const double *dz, const double *P, const double *pbhp, const double *rec,
                     const double *wi_dk, const double *lam, const double *objp, double *grad);
void launch_bsr_transpose(hipStream_t s, int nb, long nnzb, const int *tperm, const double *val,
                          double *valT);
// blocks of the convergence and update reductions (capped: few partials)
__host__ __device__ inline int conv_blocks(int n) {
    const int b = (n + kBlock - 1) / kBlock;
    return b < 2048 ? b : 2048;
}
__host__ __device__ inline int update_blocks(int n) { return conv_blocks(n); }

// ---- linear algebra kernels (fim_spmv.hip, fim_linalg.hip) -----------------
void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const double *val, const double *x, double *y, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr);
void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const float *val, const float *x, float *y, hipEvent_t e0 = nullptr,
                 hipEvent_t e1 = nullptr);
void launch_to_float(hipStream_t s, long n, const double *x, float *y);
void launch_to_double(hipStream_t s, long n, const float *x, double *y);
void launch_bj_setup(hipStream_t s, int nb, int nrows, const int *diagpos, const double *val,
                     double *dinv, int *bad);
void launch_bj_apply(hipStream_t s, int nb, int nrows, const double *dinv, const double *x,
                     double *y);
// partial-sum helpers shared by the Krylov kernels: blocks of a vector
// kernel, capped at 2048 (8 per CU) so a reduction has few partials
__host__ __device__ inline int vec_blocks(long nvec) {
    const long b = (nvec + kBlock - 1) / kBlock;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}
void launch_norm2(hipStream_t s, long nvec, const double *x, double *partials, double *out);
void launch_normalize_precond(hipStream_t s, int nb, int nrows, const double *w,
                              const double *hptr, double *v, double *z, const double *dinv);
void launch_multidot(hipStream_t s, long nvec, int nv, const double *V, const double *w,
                     double *partials, double *dst, const int *gate);
void launch_multidot(hipStream_t s, long nvec, int nv, const float *V, const float *w,
                     double *partials, double *dst, const int *gate);
// (mirror: see update_finish_body; nullptr for none)
void launch_update_norm(hipStream_t s, long nvec, int nv, const double *V, const double *coef,
                        double *w, double *partials, double *hnext, const int *gate,
                        int *reorth, double *hacc, double *mirror = nullptr);
void launch_update_norm(hipStream_t s, long nvec, int nv, const float *V, const double *coef,
                        float *w, double *partials, double *hnext, const int *gate,
                        int *reorth, double *hacc, double *mirror = nullptr);
void launch_residual(hipStream_t s, long nvec, const double *b, const double *Ax, double *r,
                     double *partials, double *out);
void launch_scale_copy(hipStream_t s, long nvec, const double *x, double a, double *y);
void launch_axpy_multi(hipStream_t s, long nvec, int k, const double *Z, const double *y,
                       double *x);
void launch_axpy_multi(hipStream_t s, long nvec, int k, const float *Z, const double *y,
                       double *x);

// ---- CPR / pressure AMG kernels (fim_amg.hip) -----------------------------------
constexpr int kCoarseMax = 64;       // cells of the level that is inverted densely
void launch_amg_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sys,
                        double *wq, double *ap);
void launch_cprT_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sysT,
                         double *wq, double *ap);
void launch_amg_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sys,
                        double *wq, float *ap);
void launch_amg_coarsen(hipStream_t s, const AmgLevel &F, const AmgLevel &C, const int *cfs_ptr,
                        const int *cfs_idx);
void launch_amg_coarsest_setup(hipStream_t s, const AmgLevel &L, double *M, double *Minv,
                               double *colk, int *bad);
void launch_amg_coarsest_solve(hipStream_t s, const AmgLevel &L, const double *Minv);

// Exact solve of a coarsest level of up to a few thousand cells by block
// elimination over slabs: the cells of one coordinate value of the axis
// (the level's longest) form a slab, the slabs couple only to their two
// neighbours through the axis's stencil entries (diagonal blocks), and every
// well lies in one slab and joins its block.  Setup: the Schur complements
// D_b = A_bb - A_b,b-1 inv(D_b-1) A_b-1,b, each inverted in place by
// Gauss-Jordan elimination; solve: forward and backward block substitution.
constexpr int kSlabMax = 96;           // unknowns of one slab (cells and wells)
constexpr int kExactCellsDefault = 4096;
constexpr int kExactGemvCols = 8192;      // columns of a dense inverse product (LDS)
constexpr int kExactSlabDoubles = 4096;   // slabs x largest block: the solve's LDS vectors
struct AmgExact {
    int axis;                  // 0 = x, 1 = y, 2 = z
    int nslab;                 // slabs (the level's extent along the axis)
    int nu, nv;                // in-slab extents: position p = u + nu * v
    int ncs;                   // cells per slab (nu * nv)
    int mmax;                  // largest block (cells and the slab's wells)
    const int *swp;            // [nslab + 1] slab -> range in sw
    const int *sw;             // wells of each slab, ascending
    const int *wrank;          // [nw] position of a well among its slab's wells
    double *binv;              // [nslab][mmax][mmax] inverted Schur complements (and
                               // kSlabMax doubles of zero padding)
    int *bad;                  // set on a zero or non-finite pivot
    double *X;                 // the level's inverse [nst][ldx]: rows in the level's
                               // storage order (padded ones zero), columns in slab order
                               // (slab b's at b * ncs + swp[b]); null: applied by
                               // substitution over the slabs in one workgroup
    const int *cmap;           // [ncol] column -> storage index
    int nst, ncol, ldx;        // 2 * half + nw; nslab * ncs + nw; row stride (even)
    int twist;                 // with X: the factorisation is two-sided, binv holding
                               // inv(D_b) below slab twist, inv(E_b) above it and the
                               // twist block's inverse at it
};
size_t exact_solve_lds(const AmgExact &E);     // dynamic LDS of the solve (bytes)
size_t exact_factor_lds(const AmgExact &E);    // and of the factorisation
hipError_t exact_allow_lds();
void launch_amg_exact_factor(hipStream_t s, const AmgLevel &L, const AmgExact &E);
void launch_amg_exact_solve(hipStream_t s, const AmgLevel &L, const AmgExact &E);
void launch_amg_exact_inverse(hipStream_t s, const AmgLevel &L, const AmgExact &E);
void launch_amg_exact_gemv(hipStream_t s, const AmgLevel &L, const AmgExact &E);
void launch_amg_sweep(hipStream_t s, const AmgLevel &L, const AmgLevel &C, int color, int mode);
void launch_amg_presmooth(hipStream_t s, const AmgLevel &L);
// seg_min: levels with at least this many entries per colour restrict by
// row segments (<= 0: never); the sums are the same bit for bit
constexpr int kSegRowsDefault = 1 << 18;
void launch_amg_restrict(hipStream_t s, const AmgLevel &F, const AmgLevel &C, long seg_min);
void launch_amg_correct(hipStream_t s, const AmgLevel &F, const AmgLevel &C);
void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const double *w, const double *hptr, double *v,
                         const double *wq);
void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const double *w, const double *hptr, float *v,
                         const double *wq);
void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const float *w, const double *hptr, float *v,
                         const double *wq);
void launch_cpr_finish(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                       const int *split0, const int *colsplit, Sys sys, const double *ap,
                       const double *v, const double *dinv, double *z);
enum { kCellsZero = 1, kCellsCorr = 2, kWellsZero = 4, kWellsCorr = 8, kWellsSnap = 16 };

// ---- block-Jacobi ILU(0) over box subdomains (fim_ilu.hip) ------------------
struct IluTiles {
    int tx, ty, tz;             // tile extents (cells)
    int ntx, nty, ntz;          // tiles per axis
    const int *rtile;           // [n+nw] subdomain of each row (wells alone: ntiles + w)
    const int *twp, *tw;        // [ntiles+1], wells joined to each tile (ascending)
    const int *wlocal;          // [nw] slot of a joined well among its tile's wells
    const int *single;          // [nsingle] wells that stand alone
    int nsingle, maxwells;      // maxwells: most wells joined to one tile
    // Sweep records of tiles whose pencils fit one workgroup (tx*ty <= 256):
    // element offset from the factors' start (a multiple of 4 elements, so
    // 16-byte aligned for float and double factors), steps tx+ty+tz-2 and
    // records (cells) per tile; poff < 0 when the tiles take the general
    // sweeps.
    long poff;
    int psteps, prec;
    long nnzb;                  // blocks of A
};
// LDS bytes of the factorisation kernel
size_t ilu_factor_lds(int nb, const IluTiles &T);
// ints of LDS the record order of a tile takes (see ilu_rank_table)
__host__ __device__ int ilu_rank_ints(const IluTiles &T);
// elements of esize bytes in the factor buffer (the factors in the layout
// of A, then the sweep records when T.poff >= 0)
size_t ilu_factor_elems(int nb, long nnzb, const IluTiles &T, int esize);
int ilu_threads(const IluTiles &T);
size_t ilu_solve_lds(int nb, const IluTiles &T);
hipError_t ilu_allow_lds(int nb, size_t bytes);
void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, double *lu,
                       int *bad);
void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, float *lu,
                       int *bad);
// right-hand side of a solve: b, or (ap set) the residual b - A x1 of the CPR
// first stage with x1 = px in level-0 AMG order, x1 added back to slot 0.
// VT: element type of b (and of the result), LT: of ap (and of the factors).
template <class VT, class LT>
struct IluRhs {
    const VT *b;
    const LT *ap;               // [nnzb][nb] pressure column of A, or null
    const int *colsplit;        // [nnzb] column -> level-0 entry
    const int *split0;          // [n] cell -> level-0 entry
    const double *px;           // level-0 iterate (cells, then wells)
    int nsplit;                 // 2*half of level 0 (first well entry)
    const double *pw = nullptr; // [n][nb] prolongation weights of the correction, or null
                                // (pressure slot only)
    int nxp = 0;                // level-0 row length of the split numbering (nx rounded
                                // up to even): a cell's neighbours' entries follow from its own
};
void launch_ilu_solve(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys,
                      const double *lu, const IluRhs<double, double> &R, double *x);
void launch_ilu_solve(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys,
                      const float *lu, const IluRhs<float, float> &R, float *x);
void launch_normalize(hipStream_t s, long nvec, const double *w, const double *hptr, double *v);
void launch_normalize(hipStream_t s, long nvec, const double *w, const double *hptr, float *v);
void launch_normalize(hipStream_t s, long nvec, const float *w, const double *hptr, float *v);

// A cycle is a sequence of phases on levels: colour sweeps, well sweeps,
// restrictions, corrections and the dense coarsest solve.  The
// coarse part of it can run as one workgroup walking a recorded phase list
// (op = kind | level << 4 | colour << 8 | mode << 12, levels relative to the
// sub-cycle's root).
enum { kOpSweep = 0, kOpWells = 1, kOpRestrict = 2, kOpCorrect = 3, kOpCoarse = 4,
       kOpPresmooth = 5 };
constexpr int kSubLevels = 8;          // levels one sub-cycle can span
constexpr int kSubOps = 4096;          // phase-list capacity
constexpr int kSubThreads = 1024;
constexpr int kFusedCellsDefault = 4096;
inline int amg_op(int kind, int level, int color = 0, int mode = 0) {
    return kind | level << 4 | color << 8 | mode << 12;
}
// LDS arrays of one sub-cycle level: doubles (x, b, acw, awc and, when they
// fit, the stencil coefficients a; -1 = left in HBM) are offsets from the
// LDS base, ints (cps, cslot, swell, scell, sps) from the end of the
// doubles.
enum { kSubX, kSubB, kSubAcw, kSubAwc, kSubA, kSubCps, kSubCslot, kSubSwell, kSubScell, kSubSps,
       kSubArrays };
struct AmgSub {
    AmgLevel lv[kSubLevels + 1];       // root first; entries past the coarsest stay empty
    int off[kSubLevels + 1][kSubArrays];
    int nlev;                          // levels from the root to the coarsest
    int ldoubles;                      // LDS doubles before the int arrays
    int opsoff;                        // phase list offset among the ints
    const int *ops;
    int nops;
    const double *Minv;                // dense inverse of the coarsest level
    int minvoff;                       // its LDS offset (doubles), -1 = read from HBM
    int rbufoff;                       // LDS offset (doubles) of the restriction's scratch
    const uint4 *img;                  // the LDS image in HBM (the levels' arrays live in it)
    int img_n16;                       // its size in 16-byte units
};
size_t amg_subcycle_lds(const AmgSub &P);          // dynamic LDS bytes of one launch
hipError_t amg_subcycle_allow_lds(size_t bytes);
hipError_t dense_allow_lds();                      // LDS of the coarsest-level inverse
void launch_amg_subcycle(hipStream_t s, const AmgSub &P);

// ---- batched launches over the members of an ensemble ------------------------
//
// One launch covers many independent reservoirs (members).  Member m takes
// the blocks [bstart[m], bstart[m+1]) of the grid; it works in the launch
// when flags[m] has the launch's bit, and its blocks exit at once otherwise.
// Inside, a member's blocks compute exactly what the member's own launch
// computes (the kernel bodies take the block index and count of the
// member's part instead of blockIdx.x / gridDim.x), so a member advanced in
// a batch is bit for bit the member advanced alone.
constexpr int kMaxLevels = 16;                      // AMG levels of one member
enum { kOnNewton = 1, kAold = 2, kOnSolve = 4, kOnCycle = 8, kOnFinish = 16, kOnUpdate = 32,
       kFirstCycle = 64 };

struct Batch {
    const int *bstart;      // [nm+1] first block of every member (device)
    const int *flags;       // [nm] what every member takes part in (device)
    int nm, bit;
};

// Everything one member's kernels read: its grid, fluid, wells and system,
// and the device buffers of its context (all owned by the member's context).
struct Member {
    Grid g;
    Phys f;
    Wells wells;
    Sys sys;
    int n, nw, nb, nrows, m;
    long nvec;
    double ds_max, dp_max;
    const double *pvref, *depth, *tx, *ty, *tz;
    double *P, *Sw, *X, *pbhp;
    int8_t *flag;
    double *rec, *aold, *wmeas, *partials, *scal;
    double *V, *Z, *w, *x, *b, *r, *t, *H, *tmp, *ydev;
    int *reorth;
    // CPR with the block-Jacobi ILU(0) second stage
    IluTiles T;
    double *lu;
    int *ilu_bad;
    int nlev;
    AmgLevel lv[kMaxLevels];
    const int *cfs_ptr[kMaxLevels], *cfs_idx[kMaxLevels];
    const int *split0, *colsplit;
    double *wq, *ap, *Mden, *Minv, *colk;
    int *amg_bad;
    int exact;              // coarsest level solved by slabs (ex), else densely (Minv)
    AmgExact ex;
    const int *ops;         // the member's whole AMG cycle, as a phase list
    int nops;
    double *rbuf;           // residuals of a restriction (2*half of level 0)
};

// the two save slots of a member's state (step start, sub-step start)
struct StateSlots {
    double *P[2], *Sw[2], *X[2], *pbhp[2];
    int8_t *flag[2];
};

// member m and its block view (b, nb) of this block of a batched launch;
// false when the member does not take part
__device__ inline bool batch_view(const Batch &B, int &m, int &b, int &nb) {
    const int bx = blockIdx.x;
    int lo = 0, hi = B.nm - 1;
    while (lo < hi) {                   // the last member whose first block is <= bx
        const int mid = (lo + hi + 1) >> 1;
        if (B.bstart[mid] <= bx) lo = mid;
        else hi = mid - 1;
    }
    m = lo;
    b = bx - B.bstart[m];
    nb = B.bstart[m + 1] - B.bstart[m];
    return (B.flags[m] & B.bit) != 0;
}

// Launchers: (stream, member table, batch, total blocks = bstart[nm]).
// The per-member block counts are those of the single launches; "one"
// batches take one block per member.  Scalar slots (slot, s_norm, s_res)
// are offsets into each member's scal array.
int blocks_for_cells(int n);
int spmv_blocks(int nb, int nrows);
int dot_groups(int nv);
int dense_lds_max();
hipError_t batch_allow_lds();
hipError_t ilu_batch_allow_lds(int nb, size_t bytes);
void launchb_props(hipStream_t s, int nb, const Member *mem, Batch B, int total);
void launchb_assemble(hipStream_t s, int nb, const Member *mem, Batch cells, int tcells,
                      Batch wells, int twells, const double *dt);
void launchb_conv(hipStream_t s, int nb, const Member *mem, Batch part, int tpart, Batch one,
                  int tone, const double *dt, int slot);
void launchb_newton_update(hipStream_t s, int nb, const Member *mem, Batch part, int tpart,
                           Batch one, int tone, int slot);
void launchb_state_copy(hipStream_t s, const Member *mem, const int *bstart, const int *flags,
                        int nm, int total, const StateSlots *slots, int k, int save_bit,
                        int restore_bit);
void launchb_gather_scalars(hipStream_t s, const Member *mem, Batch one, int tone, int first,
                            int count, double *packed, int ld);
void launchb_scale_zero(hipStream_t s, const Member *mem, Batch B, int total);
void launchb_norm_b(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one, int tone,
                    int slot);
void launchb_spmv(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j);
void launchb_multidot(hipStream_t s, const Member *mem, Batch part, int tpart, Batch sum,
                      int tsum, int j, bool second);
void launchb_update_norm(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one,
                         int tone, int j, bool second);
void launchb_hcols(hipStream_t s, const Member *mem, Batch one, int tone, int j, double *packed,
                   int ld);
void launchb_axpy(hipStream_t s, const Member *mem, Batch B, int total, const int *kcount,
                  const double *ypacked, int ld);
void launchb_residual(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one,
                      int tone, int slot);
void launchb_cpr_restrict(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j,
                          int first_bit, int s_norm, int s_res);
void launchb_amg_cycle(hipStream_t s, const Member *mem, Batch one, int tone, size_t exact_lds);
void launchb_amg_extract(hipStream_t s, int nb, const Member *mem, Batch B, int total);
void launchb_amg_coarsen(hipStream_t s, const Member *mem, Batch B, int total, int level);
void launchb_amg_coarsest(hipStream_t s, const Member *mem, Batch one, int tone, int nmax,
                          size_t exact_lds);
void launchb_ilu_factor(hipStream_t s, int nb, const Member *mem, Batch B, int total, int threads,
                        size_t lds);
void launchb_ilu_solve(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j,
                       int threads, size_t lds);

}  // namespace fim
