// fim_ilu.hip - block-Jacobi ILU(0) over box subdomains (paper Sec. 5.1:
// block Jacobi over subdomains with ILU(0) inside each, used as the
// smoother of CPR and on its own).
//
// A subdomain ("tile") is a box of tx x ty x tz cells plus every well whose
// perforations all lie in it; other wells stand alone.  Inside a tile the
// factorisation is the natural-order block ILU(0) of the tile's diagonal
// part of A (couplings to other tiles dropped): L_ik = A_ik inv(U_kk), then
// A_ij -= L_ik U_kj for the (i, j) of the pattern, the inverted pivot block
// kept in the diagonal slot.  With one tile covering the grid it is the
// plain natural-order BILU(0).
//
// On a 7-point stencil row i depends only on rows in the previous
// hyperplane li + lj + lk - 1 of its tile (and a well row on all of its
// cells), so one workgroup per tile walks the hyperplanes with a barrier
// between them; tiles run in parallel.  The triangular solves walk a row's
// blocks in the pattern's canonical order (-z, -y, -x, diagonal, +x, +y,
// +z, then wells), so neighbours are found from the row's own position,
// and keep the tile's vector in LDS.
#include <math.h>

#include "fim_block.h"
#include "fim_internal.h"

namespace fim {

struct TileBox {
    int i0, j0, k0, txe, tye, tze;   // origin and extents (clipped at the grid edge)
};

__device__ inline TileBox tile_box(const Grid &g, const IluTiles &T, int b) {
    TileBox t;
    const int bi = b % T.ntx, bj = (b / T.ntx) % T.nty, bk = b / (T.ntx * T.nty);
    t.i0 = bi * T.tx;
    t.j0 = bj * T.ty;
    t.k0 = bk * T.tz;
    t.txe = min(T.tx, g.nx - t.i0);
    t.tye = min(T.ty, g.ny - t.j0);
    t.tze = min(T.tz, g.nz - t.k0);
    return t;
}

// Copy of A's blocks [q0, q1) into lu by the whole workgroup (contiguous,
// 16-byte accesses).
template <class LT>
__device__ inline void copy_blocks(const double *__restrict__ val, LT *__restrict__ lu, long q0,
                                   long q1, int b2) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const long e0 = q0 * b2, e1 = q1 * b2;        // element range
    long e = e0 + threadIdx.x * 2;
    if (e0 & 1) {                                  // odd start: one scalar first
        if (threadIdx.x == 0) lu[e0] = (LT)val[e0];
        e = e0 + 1 + threadIdx.x * 2;
    }
    for (; e + 1 < e1; e += 2L * blockDim.x) {
        const d2v v = *reinterpret_cast<const d2v *>(val + e);
        lu[e] = (LT)v.x;
        lu[e + 1] = (LT)v.y;
    }
    if (e < e1) lu[e] = (LT)val[e];
}

// ILU(0) of one row in place (lu holds A's values for the row on entry):
// IKJ form restricted to the row's tile.  The row's lower neighbours in its
// tile are factored already.
template <int NB, class LT>
__device__ void factor_row(int row, const IluTiles &T, const Sys &sys, LT *lu, int *bad) {
    constexpr int B2 = NB * NB;
    const int t = T.rtile[row];
    const int b0 = sys.rowptr[row], b1 = sys.rowptr[row + 1];
    for (int qk = b0; qk < b1; ++qk) {
        const int k = sys.colind[qk];
        if (k >= row) break;
        if (T.rtile[k] != t) continue;
        double a[B2], u[B2], l[B2];
#pragma unroll
        for (int e = 0; e < B2; ++e) {
            a[e] = (double)lu[(size_t)qk * B2 + e];
            u[e] = (double)lu[(size_t)sys.diagpos[k] * B2 + e];
        }
        block_mul<NB>(a, u, l);
#pragma unroll
        for (int e = 0; e < B2; ++e) lu[(size_t)qk * B2 + e] = (LT)l[e];
        const int k0 = sys.rowptr[k], k1 = sys.rowptr[k + 1];
        for (int qj = qk + 1; qj < b1; ++qj) {
            const int j = sys.colind[qj];
            if (T.rtile[j] != t) continue;
            for (int qkj = k0; qkj < k1; ++qkj) {
                if (sys.colind[qkj] != j) continue;
                double ukj[B2], p[B2];
#pragma unroll
                for (int e = 0; e < B2; ++e) ukj[e] = (double)lu[(size_t)qkj * B2 + e];
                block_mul<NB>(l, ukj, p);
#pragma unroll
                for (int e = 0; e < B2; ++e)
                    lu[(size_t)qj * B2 + e] = (LT)((double)lu[(size_t)qj * B2 + e] - p[e]);
            }
        }
    }
    const int di = sys.diagpos[row];
    double d[B2], inv[B2];
#pragma unroll
    for (int e = 0; e < B2; ++e) d[e] = (double)lu[(size_t)di * B2 + e];
    if (!invert_block<NB>(d, inv)) {
        *bad = 1;
#pragma unroll
        for (int e = 0; e < B2; ++e) inv[e] = (e % (NB + 1) == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < B2; ++e) lu[(size_t)di * B2 + e] = (LT)inv[e];
}

// The same factorisation for a cell row without well columns, found from
// the row's position: on a 7-point pattern the only entry ILU(0) changes
// besides the lower blocks is the diagonal, D_i = A_ii - sum_k L_ik U_ki
// over the lower neighbours k of the tile (in column order -z, -y, -x),
// with U_ki the +z / +y / +x block of row k.  Returns false (nothing done)
// for rows with well columns.
template <int NB, class LT>
__device__ bool factor_cell_row(int i, int j, int k, const Grid &g, const IluTiles &T,
                                const TileBox &tb, const Sys &sys, LT *lu, int *bad) {
    constexpr int B2 = NB * NB;
    const int r = i + g.nx * (j + g.ny * k);
    const int q0 = sys.rowptr[r];
    const int nlow = (k > 0) + (j > 0) + (i > 0);
    const int nup = (i + 1 < g.nx) + (j + 1 < g.ny) + (k + 1 < g.nz);
    if (sys.rowptr[r + 1] - q0 != nlow + 1 + nup) return false;
    const int qd = q0 + nlow;
    double d[B2];
#pragma unroll
    for (int e = 0; e < B2; ++e) d[e] = (double)lu[(size_t)qd * B2 + e];
    const int li = i - tb.i0, lj = j - tb.j0, lk = k - tb.k0;
    // lower neighbours in column order; for each: its row index, the
    // position of its diagonal and of its block towards row r
    int qk = q0;
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const bool exists = dir == 0 ? k > 0 : (dir == 1 ? j > 0 : i > 0);
        if (!exists) continue;
        const bool in = dir == 0 ? lk > 0 : (dir == 1 ? lj > 0 : li > 0);
        if (in) {
            const int ki = i - (dir == 2), kj = j - (dir == 1), kk = k - (dir == 0);
            const int rk = r - (dir == 0 ? g.nx * g.ny : (dir == 1 ? g.nx : 1));
            const int qdk = sys.rowptr[rk] + (kk > 0) + (kj > 0) + (ki > 0);
            // U_ki: +x, +y or +z block of row k
            const int qki = qdk + 1 + (dir <= 1 ? (ki + 1 < g.nx) : 0) + (dir == 0 ? (kj + 1 < g.ny) : 0);
            double a[B2], u[B2], l[B2], uk[B2], p[B2];
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                a[e] = (double)lu[(size_t)qk * B2 + e];
                u[e] = (double)lu[(size_t)qdk * B2 + e];
            }
            block_mul<NB>(a, u, l);
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                lu[(size_t)qk * B2 + e] = (LT)l[e];
                uk[e] = (double)lu[(size_t)qki * B2 + e];
            }
            block_mul<NB>(l, uk, p);
#pragma unroll
            for (int e = 0; e < B2; ++e) d[e] -= p[e];
        }
        ++qk;
    }
    double inv[B2];
    if (!invert_block<NB>(d, inv)) {
        *bad = 1;
#pragma unroll
        for (int e = 0; e < B2; ++e) inv[e] = (e % (NB + 1) == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < B2; ++e) lu[(size_t)qd * B2 + e] = (LT)inv[e];
    return true;
}

// inverse of the diagonal block of a row that is a subdomain of its own
template <int NB, class LT>
__device__ void factor_alone(int row, const Sys &sys, LT *lu, int *bad) {
    constexpr int B2 = NB * NB;
    const int di = sys.diagpos[row];
    double d[B2], inv[B2];
#pragma unroll
    for (int e = 0; e < B2; ++e) d[e] = (double)lu[(size_t)di * B2 + e];
    if (!invert_block<NB>(d, inv)) {
        *bad = 1;
#pragma unroll
        for (int e = 0; e < B2; ++e) inv[e] = (e % (NB + 1) == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < B2; ++e) lu[(size_t)di * B2 + e] = (LT)inv[e];
}

// One workgroup per tile, then one for the wells that stand alone.  The
// tile's rows (cells and its wells) are copied from A first, each x-row of
// the tile being one contiguous run of blocks.
template <int NB, class LT>
__global__ __launch_bounds__(256) void k_ilu_factor(Grid g, IluTiles T, Sys sys, LT *lu,
                                                    int *bad) {
    constexpr int B2 = NB * NB;
    const int b = blockIdx.x;
    const int ntiles = T.ntx * T.nty * T.ntz;
    if (b >= ntiles) {
        for (int e = 0; e < T.nsingle; ++e) {
            const int r = g.n + T.single[e];
            copy_blocks(sys.val, lu, sys.rowptr[r], sys.rowptr[r + 1], B2);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < T.nsingle; e += blockDim.x)
            factor_alone<NB, LT>(g.n + T.single[e], sys, lu, bad);
        return;
    }
    const TileBox tb = tile_box(g, T, b);
    for (int seg = 0; seg < tb.tye * tb.tze; ++seg) {
        const int j = tb.j0 + seg % tb.tye, k = tb.k0 + seg / tb.tye;
        const int r0 = tb.i0 + g.nx * (j + g.ny * k);
        copy_blocks(sys.val, lu, sys.rowptr[r0], sys.rowptr[r0 + tb.txe], B2);
    }
    for (int e = T.twp[b]; e < T.twp[b + 1]; ++e) {
        const int r = g.n + T.tw[e];
        copy_blocks(sys.val, lu, sys.rowptr[r], sys.rowptr[r + 1], B2);
    }
    __syncthreads();
    const int nlev = tb.txe + tb.tye + tb.tze - 2;
    for (int s = 0; s < nlev; ++s) {
        for (int p = threadIdx.x; p < tb.txe * tb.tye; p += blockDim.x) {
            const int li = p % tb.txe, lj = p / tb.txe, lk = s - li - lj;
            if (lk < 0 || lk >= tb.tze) continue;
            const int i = tb.i0 + li, j = tb.j0 + lj, k = tb.k0 + lk;
            if (!factor_cell_row<NB, LT>(i, j, k, g, T, tb, sys, lu, bad))
                factor_row<NB, LT>(i + g.nx * (j + g.ny * k), T, sys, lu, bad);
        }
        __syncthreads();
    }
    for (int e = T.twp[b] + threadIdx.x; e < T.twp[b + 1]; e += blockDim.x)
        factor_row<NB, LT>(g.n + T.tw[e], T, sys, lu, bad);
}

// acc -= blk * v (block-vector product summed first, as a matrix-vector
// product would)
template <int NB, class BT>
__device__ inline void sub_mv(double (&acc)[NB], const BT *blk, const double *v) {
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        double t = (double)blk[r * NB] * v[0];
#pragma unroll
        for (int c = 1; c < NB; ++c) t += (double)blk[r * NB + c] * v[c];
        acc[r] -= t;
    }
}

template <int NB>
struct Blk {
    double v[NB * NB];
};

template <int NB, class LT>
__device__ inline void load_blk(Blk<NB> &dst, const LT *src) {
#pragma unroll
    for (int e = 0; e < NB * NB; ++e) dst.v[e] = (double)src[e];
}

// Right-hand side of row r: b, or for the CPR second stage the residual
// v - A x1 of the first stage (A x1 from the compact pressure column, x1
// the level-0 pressure correction), whose correction corr(r) is added to the
// first slot of the result.
// (the first eight blocks of the row issue their loads together; longer
// rows, of perforated cells and wells, finish in a loop)
template <int NB, class RT>
__device__ inline void rhs_row(const RT &R, const Sys &sys, int r, double (&acc)[NB],
                               int q0 = -1) {
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = (double)R.b[(size_t)r * NB + u];
    if (!R.ap) return;
    if (q0 < 0) q0 = sys.rowptr[r];
    const int q1 = sys.rowptr[r + 1];
    constexpr int K = 8;
    // a slot past the row's end loads the row's last block (every row has
    // one) and is dropped by a select: no branch between the loads
    int cs[K];
    double a[K][NB];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = min(q0 + k, q1 - 1);
        cs[k] = R.colsplit[q];
#pragma unroll
        for (int u = 0; u < NB; ++u) a[k][u] = (double)R.ap[(size_t)q * NB + u];
    }
    double p[K];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = R.px[cs[k]];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool on = q0 + k < q1;
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] -= (on ? a[k][u] : 0.0) * (on ? p[k] : 0.0);
    }
    for (int q = q0 + K; q < q1; ++q) {
        const double pq = R.px[R.colsplit[q]];
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] -= (double)R.ap[(size_t)q * NB + u] * pq;
    }
}

// the first-stage correction in component u of row r: the pressure slot,
// or every component scaled by the prolongation weights pw of its cell
template <int NB, class RT>
__device__ inline double rhs_corr(const RT &R, int n, int r, int u) {
    if (!R.ap) return 0.0;
    const double mu = r < n ? R.px[R.split0[r]] : R.px[R.nsplit + (r - n)];
    if (R.pw && r < n) return R.pw[(size_t)r * NB + u] * mu;
    return u == 0 ? mu : 0.0;
}

// The tile's wells, between the forward and backward sweeps over its cells:
// forward over their perforated cells (all in the tile), then x = inv(U) y
// (well rows have no upper part).
template <int NB, class LT, class RT>
__device__ void solve_tile_wells(const Grid &g, const TileBox &tb, const Sys &sys,
                                 const LT *lu, const RT &R, double *y, const IluTiles &T,
                                 int w0, int nwt, int ncell) {
    constexpr int B2 = NB * NB;
    const int n = g.n;
    for (int e = threadIdx.x; e < nwt; e += blockDim.x) {
        const int r = n + T.tw[w0 + e];
        double acc[NB];
        rhs_row<NB>(R, sys, r, acc);
        for (int q = sys.rowptr[r]; q < sys.rowptr[r + 1]; ++q) {
            const int col = sys.colind[q];
            if (col >= n) break;
            const int ci = col % g.nx, cj = (col / g.nx) % g.ny, ck = col / (g.nx * g.ny);
            const int lc = (ci - tb.i0) + tb.txe * ((cj - tb.j0) + tb.tye * (ck - tb.k0));
            sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)lc * NB);
        }
        double xw[NB] = {};
        sub_mv<NB>(xw, lu + (size_t)sys.diagpos[r] * B2, acc);
#pragma unroll
        for (int u = 0; u < NB; ++u) y[(size_t)(ncell + e) * NB + u] = -xw[u];
    }
}

// Both sweeps over the cells of a tile whose (li, lj) pencils fit the
// workgroup: thread (li, lj) owns the pencil and meets its cells in order
// of lk, one per hyperplane, so it loads the blocks of its next kAhead
// cells while the hyperplanes before them are solved.  Row starts and the
// right side are staged in LDS first.  Same arithmetic, same order, as the
// general sweeps.
template <int NB, class LT, class RT>
__device__ void solve_cells_pencils(const Grid &g, const TileBox &tb, const Sys &sys,
                                    const LT *__restrict__ lu, const RT &R,
                                    double *y, int *rp, const IluTiles &T, int blk, int w0, int nwt,
                                    int ncell) {
    constexpr int B2 = NB * NB;
    constexpr int kAhead = 2;                     // deeper costs occupancy (VGPRs)
    const int sxy = tb.txe * tb.tye;
    // two rows per thread at a time so their loads overlap
    for (int l0 = threadIdx.x; l0 < ncell; l0 += 2 * blockDim.x) {
        int rr[2], q0[2];
        bool on[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = l0 + h * blockDim.x;
            on[h] = l < ncell;
            const int li = l % tb.txe, lj = (l / tb.txe) % tb.tye, lk = l / sxy;
            rr[h] = on[h] ? (tb.i0 + li) + g.nx * ((tb.j0 + lj) + g.ny * (tb.k0 + lk)) : 0;
            q0[h] = on[h] ? sys.rowptr[rr[h]] : 0;
        }
        double acc[2][NB];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (on[h]) rhs_row<NB>(R, sys, rr[h], acc[h], q0[h]);
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (on[h]) {
                const int l = l0 + h * blockDim.x;
                rp[l] = q0[h];
#pragma unroll
                for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = acc[h][u];
            }
    }
    __syncthreads();
    const bool own = (int)threadIdx.x < sxy;
    const int li = threadIdx.x % tb.txe, lj = threadIdx.x / tb.txe;
    const int i = tb.i0 + li, j = tb.j0 + lj;
    const int nlev = tb.txe + tb.tye + tb.tze - 2;
    // forward: lower blocks -z, -y, -x of cell lk
    auto lower = [&](int lk, Blk<NB> &bz, Blk<NB> &by, Blk<NB> &bx) {
        const int k = tb.k0 + lk;
        const int q = rp[li + tb.txe * (lj + tb.tye * lk)];
        const int qy = q + (k > 0), qx = qy + (j > 0);
        if (lk > 0) load_blk<NB>(bz, lu + (size_t)q * B2);
        if (lj > 0) load_blk<NB>(by, lu + (size_t)qy * B2);
        if (li > 0) load_blk<NB>(bx, lu + (size_t)qx * B2);
    };
    // blocks of the next kAhead cells of the pencil, in flight
    Blk<NB> fz[kAhead], fy[kAhead], fx[kAhead];
    if (own)
#pragma unroll
        for (int a = 0; a < kAhead; ++a)
            if (a < tb.tze) lower(a, fz[a], fy[a], fx[a]);
    for (int s = 0; s < nlev; ++s) {
        const int lk = s - li - lj;
        if (own && lk >= 0 && lk < tb.tze) {
            const int l = li + tb.txe * (lj + tb.tye * lk);
            double acc[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) acc[u] = y[(size_t)l * NB + u];
            if (lk > 0) sub_mv<NB>(acc, fz[0].v, y + (size_t)(l - sxy) * NB);
            if (lj > 0) sub_mv<NB>(acc, fy[0].v, y + (size_t)(l - tb.txe) * NB);
            if (li > 0) sub_mv<NB>(acc, fx[0].v, y + (size_t)(l - 1) * NB);
#pragma unroll
            for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = acc[u];
#pragma unroll
            for (int a = 0; a + 1 < kAhead; ++a) {
                fz[a] = fz[a + 1];
                fy[a] = fy[a + 1];
                fx[a] = fx[a + 1];
            }
            if (lk + kAhead < tb.tze) lower(lk + kAhead, fz[kAhead - 1], fy[kAhead - 1], fx[kAhead - 1]);
        }
        __syncthreads();
    }
    solve_tile_wells<NB, LT>(g, tb, sys, lu, R, y, T, w0, nwt, ncell);
    __syncthreads();
    // backward: +x, +y, +z blocks and the inverted diagonal of cell lk
    auto upper = [&](int lk, Blk<NB> &ux, Blk<NB> &uy, Blk<NB> &uz, Blk<NB> &dd) {
        const int k = tb.k0 + lk;
        const int qd = rp[li + tb.txe * (lj + tb.tye * lk)] + (k > 0) + (j > 0) + (i > 0);
        const int qy = qd + 1 + (i + 1 < g.nx), qz = qy + (j + 1 < g.ny);
        load_blk<NB>(dd, lu + (size_t)qd * B2);
        if (li + 1 < tb.txe) load_blk<NB>(ux, lu + (size_t)(qd + 1) * B2);
        if (lj + 1 < tb.tye) load_blk<NB>(uy, lu + (size_t)qy * B2);
        if (lk + 1 < tb.tze) load_blk<NB>(uz, lu + (size_t)qz * B2);
    };
    Blk<NB> gx[kAhead], gy[kAhead], gz[kAhead], gd[kAhead];
    if (own)
#pragma unroll
        for (int a = 0; a < kAhead; ++a)
            if (a < tb.tze) upper(tb.tze - 1 - a, gx[a], gy[a], gz[a], gd[a]);
    for (int s = nlev - 1; s >= 0; --s) {
        const int lk = s - li - lj;
        if (own && lk >= 0 && lk < tb.tze) {
            const int k = tb.k0 + lk;
            const int r = i + g.nx * (j + g.ny * k), l = li + tb.txe * (lj + tb.tye * lk);
            double acc[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) acc[u] = y[(size_t)l * NB + u];
            if (li + 1 < tb.txe) sub_mv<NB>(acc, gx[0].v, y + (size_t)(l + 1) * NB);
            if (lj + 1 < tb.tye) sub_mv<NB>(acc, gy[0].v, y + (size_t)(l + tb.txe) * NB);
            if (lk + 1 < tb.tze) sub_mv<NB>(acc, gz[0].v, y + (size_t)(l + sxy) * NB);
            // well columns (perforated cells): the wells of this tile
            const int qw = rp[l] + (k > 0) + (j > 0) + (i > 0) + 1 + (i + 1 < g.nx) + (j + 1 < g.ny) +
                           (k + 1 < g.nz);
            for (int q = qw; q < sys.rowptr[r + 1]; ++q) {
                const int w = sys.colind[q] - g.n;
                if (T.rtile[g.n + w] == blk)
                    sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(ncell + T.wlocal[w]) * NB);
            }
            double xr[NB] = {};
            sub_mv<NB>(xr, gd[0].v, acc);
#pragma unroll
            for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = -xr[u];
#pragma unroll
            for (int a = 0; a + 1 < kAhead; ++a) {
                gx[a] = gx[a + 1];
                gy[a] = gy[a + 1];
                gz[a] = gz[a + 1];
                gd[a] = gd[a + 1];
            }
            if (lk - kAhead >= 0)
                upper(lk - kAhead, gx[kAhead - 1], gy[kAhead - 1], gz[kAhead - 1], gd[kAhead - 1]);
        }
        __syncthreads();
    }
}

// x = M^-1 rhs: forward (L y = rhs, L unit lower) and backward (U x = y)
// inside every tile; for the CPR second stage the first-stage correction is
// added to the first slot of every row of x.
template <int NB, class LT, class VT>
__global__ __launch_bounds__(256) void k_ilu_solve(Grid g, IluTiles T, Sys sys,
                                                   const LT *__restrict__ lu, IluRhs<VT, LT> R,
                                                   VT *__restrict__ x) {
    constexpr int B2 = NB * NB;
    extern __shared__ double y[];
    const int blk = blockIdx.x;
    const int ntiles = T.ntx * T.nty * T.ntz;
    const int n = g.n;
    if (blk >= ntiles) {
        for (int e = threadIdx.x; e < T.nsingle; e += blockDim.x) {
            const int r = n + T.single[e];
            double rhs[NB], acc[NB] = {};
            rhs_row<NB>(R, sys, r, rhs);
            sub_mv<NB>(acc, lu + (size_t)sys.diagpos[r] * B2, rhs);
#pragma unroll
            for (int u = 0; u < NB; ++u) x[(size_t)r * NB + u] = (VT)(-acc[u] + rhs_corr<NB>(R, n, r, u));
        }
        return;
    }
    const TileBox tb = tile_box(g, T, blk);
    const int sxy = tb.txe * tb.tye, ncell = sxy * tb.tze;
    const int w0 = T.twp[blk], nwt = T.twp[blk + 1] - w0;
    const int nlev = tb.txe + tb.tye + tb.tze - 2;
    if (sxy <= (int)blockDim.x) {
        solve_cells_pencils<NB, LT>(g, tb, sys, lu, R, y, reinterpret_cast<int *>(y + (size_t)(ncell + T.maxwells) * NB),
                                T, blk, w0, nwt, ncell);
    } else {
    // forward over the hyperplanes
    for (int s = 0; s < nlev; ++s) {
        for (int p = threadIdx.x; p < sxy; p += blockDim.x) {
            const int li = p % tb.txe, lj = p / tb.txe, lk = s - li - lj;
            if (lk < 0 || lk >= tb.tze) continue;
            const int i = tb.i0 + li, j = tb.j0 + lj, k = tb.k0 + lk;
            const int r = i + g.nx * (j + g.ny * k), l = li + tb.txe * (lj + tb.tye * lk);
            double acc[NB];
            rhs_row<NB>(R, sys, r, acc);
            int q = sys.rowptr[r];
            if (k > 0) {
                if (lk > 0) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l - sxy) * NB);
                ++q;
            }
            if (j > 0) {
                if (lj > 0) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l - tb.txe) * NB);
                ++q;
            }
            if (i > 0 && li > 0) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l - 1) * NB);
#pragma unroll
            for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = acc[u];
        }
        __syncthreads();
    }
    solve_tile_wells<NB, LT>(g, tb, sys, lu, R, y, T, w0, nwt, ncell);
    __syncthreads();
    // backward over the hyperplanes
    for (int s = nlev - 1; s >= 0; --s) {
        for (int p = threadIdx.x; p < sxy; p += blockDim.x) {
            const int li = p % tb.txe, lj = p / tb.txe, lk = s - li - lj;
            if (lk < 0 || lk >= tb.tze) continue;
            const int i = tb.i0 + li, j = tb.j0 + lj, k = tb.k0 + lk;
            const int r = i + g.nx * (j + g.ny * k), l = li + tb.txe * (lj + tb.tye * lk);
            double acc[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) acc[u] = y[(size_t)l * NB + u];
            const int qd = sys.rowptr[r] + (k > 0) + (j > 0) + (i > 0);
            int q = qd + 1;
            if (i + 1 < g.nx) {
                if (li + 1 < tb.txe) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l + 1) * NB);
                ++q;
            }
            if (j + 1 < g.ny) {
                if (lj + 1 < tb.tye) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l + tb.txe) * NB);
                ++q;
            }
            if (k + 1 < g.nz) {
                if (lk + 1 < tb.tze) sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(l + sxy) * NB);
                ++q;
            }
            for (; q < sys.rowptr[r + 1]; ++q) {
                const int w = sys.colind[q] - n;
                if (T.rtile[n + w] == blk)
                    sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(ncell + T.wlocal[w]) * NB);
            }
            double xr[NB] = {};
            sub_mv<NB>(xr, lu + (size_t)qd * B2, acc);
#pragma unroll
            for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = -xr[u];
        }
        __syncthreads();
    }
    }
    for (int l = threadIdx.x; l < ncell + nwt; l += blockDim.x) {
        int r;
        if (l < ncell) {
            const int li = l % tb.txe, lj = (l / tb.txe) % tb.tye, lk = l / sxy;
            r = (tb.i0 + li) + g.nx * ((tb.j0 + lj) + g.ny * (tb.k0 + lk));
        } else {
            r = n + T.tw[w0 + (l - ncell)];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
            x[(size_t)r * NB + u] = (VT)(y[(size_t)l * NB + u] + rhs_corr<NB>(R, n, r, u));
    }
}

// v = w / h for a new Arnoldi vector (zero when h is not a positive number)
template <class WT, class VT>
__global__ __launch_bounds__(kBlock) void k_normalize(long nvec, const WT *__restrict__ w,
                                                      const double *__restrict__ hptr,
                                                      VT *__restrict__ v) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nvec) return;
    const double h = *hptr;
    v[e] = (VT)((h > 0.0 && isfinite(h)) ? (double)w[e] / h : 0.0);
}

// ---------------------------------------------------------------------------
// launchers

template <class LT>
static void ilu_factor_impl(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, LT *lu,
                            int *bad) {
    const int nblk = T.ntx * T.nty * T.ntz + (T.nsingle > 0 ? 1 : 0);
    const int bs = ilu_threads(T);
    if (nb == 2) hipLaunchKernelGGL((k_ilu_factor<2, LT>), dim3(nblk), dim3(bs), 0, s, g, T, sys, lu, bad);
    else hipLaunchKernelGGL((k_ilu_factor<3, LT>), dim3(nblk), dim3(bs), 0, s, g, T, sys, lu, bad);
}

void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, double *lu,
                       int *bad) {
    ilu_factor_impl(s, nb, g, T, sys, lu, bad);
}

void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, float *lu,
                       int *bad) {
    ilu_factor_impl(s, nb, g, T, sys, lu, bad);
}

int ilu_threads(const IluTiles &T) {
    const int pairs = T.tx * T.ty;
    return pairs >= 256 ? 256 : ((pairs + 63) / 64) * 64;
}

size_t ilu_solve_lds(int nb, const IluTiles &T) {
    // the tile's vector, then its row starts (pencil sweeps)
    return (size_t)(T.tx * T.ty * T.tz + T.maxwells) * nb * sizeof(double) +
           (size_t)T.tx * T.ty * T.tz * sizeof(int);
}

template <class LT, class VT>
static hipError_t allow_lds_impl(int nb, size_t bytes) {
    if (nb == 2)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_solve<2, LT, VT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_solve<3, LT, VT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t ilu_allow_lds(int nb, size_t bytes) {
    hipError_t e = allow_lds_impl<double, double>(nb, bytes);
    if (e == hipSuccess) e = allow_lds_impl<float, float>(nb, bytes);
    return e;
}

template <class LT, class VT>
static void ilu_solve_impl(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys,
                           const LT *lu, const IluRhs<VT, LT> &R, VT *x) {
    const int nblk = T.ntx * T.nty * T.ntz + (T.nsingle > 0 ? 1 : 0);
    const int bs = ilu_threads(T);
    const size_t lds = ilu_solve_lds(nb, T);
    if (nb == 2)
        hipLaunchKernelGGL((k_ilu_solve<2, LT, VT>), dim3(nblk), dim3(bs), lds, s, g, T, sys, lu, R, x);
    else
        hipLaunchKernelGGL((k_ilu_solve<3, LT, VT>), dim3(nblk), dim3(bs), lds, s, g, T, sys, lu, R, x);
}

void launch_ilu_solve(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys,
                      const double *lu, const IluRhs<double, double> &R, double *x) {
    ilu_solve_impl(s, nb, g, T, sys, lu, R, x);
}

void launch_ilu_solve(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys,
                      const float *lu, const IluRhs<float, float> &R, float *x) {
    ilu_solve_impl(s, nb, g, T, sys, lu, R, x);
}

template <class WT, class VT>
static void normalize_impl(hipStream_t s, long nvec, const WT *w, const double *hptr, VT *v) {
    hipLaunchKernelGGL((k_normalize<WT, VT>), dim3((unsigned)((nvec + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, nvec, w, hptr, v);
}

void launch_normalize(hipStream_t s, long nvec, const double *w, const double *hptr, double *v) {
    normalize_impl(s, nvec, w, hptr, v);
}

void launch_normalize(hipStream_t s, long nvec, const double *w, const double *hptr, float *v) {
    normalize_impl(s, nvec, w, hptr, v);
}

void launch_normalize(hipStream_t s, long nvec, const float *w, const double *hptr, float *v) {
    normalize_impl(s, nvec, w, hptr, v);
}

}  // namespace fim
