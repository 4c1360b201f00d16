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
#include "fim_reduce.h"

namespace fim {

// Third word of a raw buffer resource on this architecture (32-bit data,
// no swizzle).  Its range check gives zeros for loads and drops stores at
// or past num_records, without a memory access: the sweeps and the
// factorisation use that for lanes without a row at a step.
constexpr int kBufferWord3 = 0x00020000;
typedef unsigned int bu2 __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, kBufferWord3);
}
__device__ inline double buf_ld(__amdgpu_buffer_rsrc_t rs, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
}
template <class LT>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t rs, int off, double v) {
    if constexpr (sizeof(LT) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu2, v), rs, off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)v), rs, off, 0, 0);
}

// (the sweeps and the pencil factorisation exchange values through LDS
// alone: lds_barrier, from fim_reduce.h)

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

// elements of a record of nblk blocks, rounded to whole 16-byte chunks
__host__ __device__ constexpr int rec_elems(int nblk, int nb, int esize) {
    return (nblk * nb * nb + 16 / esize - 1) / (16 / esize) * (16 / esize);
}

// Element index of the first chunk, and the chunk stride in elements, of
// the records (ne elements, w per chunk) of cell (li, lj) at step s;
// element j is at start + (j / w) * stride + j % w.
struct RecPos {
    int start, stride;
};
__device__ inline RecPos rec_pos(const IluTiles &T, const int *roff, int s, int li, int lj, int ne,
                                 int w) {
    const int *cnt = roff + T.psteps * T.ty, *first = cnt + T.psteps;
    const int c = cnt[s], f = first[s];
    return RecPos{f * ne + (roff[s * T.ty + lj] + li - f) * w, c * w};
}
__device__ inline int rec_at(const RecPos &p, int j, int w) {
    return p.start + (j / w) * p.stride + j % w;
}

// The same factorisation for a cell row, found from the row's position and
// read from A's values at A (A itself, or the row's copy in lu): on a
// 7-point pattern
// ILU(0) changes, besides the lower blocks L_ik = A_ik inv(U_kk), only the
// diagonal, D_i = A_ii - sum_k L_ik U_ki over the lower neighbours k of the
// tile (in column order -z, -y, -x; U_ki the +z / +y / +x block of row k,
// A's own), and the columns of wells of the tile that perforate both i and
// k, A_iw -= L_ik U_kw.  The upper blocks are A's.  The row's blocks go to
// lu (couplings leaving the tile unchanged) and, when lo / up are given,
// to the tile's sweep records at pl / pu.
template <int NB, class LT, class ST>
__device__ void factor_cell_row(int i, int j, int k, const Grid &g, const IluTiles &T,
                                const TileBox &tb, int tile, const Sys &sys, const ST *A, LT *lu,
                                int *bad, LT *lo = nullptr, LT *up = nullptr, RecPos pl = {},
                                RecPos pu = {}) {
    constexpr int W = 16 / sizeof(LT);
    constexpr int B2 = NB * NB;
    const int r = i + g.nx * (j + g.ny * k);
    const int q0 = sys.rowptr[r], q1 = sys.rowptr[r + 1];
    const int nlow = (k > 0) + (j > 0) + (i > 0);
    const int nup = (i + 1 < g.nx) + (j + 1 < g.ny) + (k + 1 < g.nz);
    const int qd = q0 + nlow;
    double d[B2];
#pragma unroll
    for (int e = 0; e < B2; ++e) d[e] = (double)A[(size_t)qd * B2 + e];
    const int li = i - tb.i0, lj = j - tb.j0, lk = k - tb.k0;
    {
        // upper blocks: A's, into lu and (zero where the neighbour lies
        // outside the tile) into the sweep record
        const int qux = qd + 1, quy = qux + (i + 1 < g.nx), quz = quy + (j + 1 < g.ny);
        const bool ex[3] = {i + 1 < g.nx, j + 1 < g.ny, k + 1 < g.nz};
        const bool hin[3] = {li + 1 < tb.txe, lj + 1 < tb.tye, lk + 1 < tb.tze};
        const int qu[3] = {qux, quy, quz};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                const double v = (double)A[(size_t)(ex[m] ? qu[m] : qd) * B2 + e];
                if (ex[m]) lu[(size_t)qu[m] * B2 + e] = (LT)v;
                if (up) up[rec_at(pu, (m + 1) * B2 + e, W)] = hin[m] ? (LT)v : (LT)0;
            }
        }
    }
    // the row's well columns (perforated cells): A's values, updated below
    // for wells of this tile
    const int qw0 = qd + 1 + nup;
    for (int q = qw0; q < q1; ++q)
#pragma unroll
        for (int e = 0; e < B2; ++e) lu[(size_t)q * B2 + e] = (LT)A[(size_t)q * B2 + e];
    // lower neighbours in column order; for each: its row index, the
    // position of its diagonal and of its block towards row r
    int qk = q0;
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        const bool exists = dir == 0 ? k > 0 : (dir == 1 ? j > 0 : i > 0);
        const bool in = dir == 0 ? lk > 0 : (dir == 1 ? lj > 0 : li > 0);
        if (lo && !in)
#pragma unroll
            for (int e = 0; e < B2; ++e) lo[rec_at(pl, dir * B2 + e, W)] = (LT)0;
        if (!exists) continue;
        if (in) {
            const int ki = i - (dir == 2), kj = j - (dir == 1), kk = k - (dir == 0);
            const int rk = r - (dir == 0 ? g.nx * g.ny : (dir == 1 ? g.nx : 1));
            const int qk0 = sys.rowptr[rk];
            const int qdk = qk0 + (kk > 0) + (kj > 0) + (ki > 0);
            // U_ki: +x, +y or +z block of row k (A's)
            const int qki = qdk + 1 + (dir <= 1 ? (ki + 1 < g.nx) : 0) + (dir == 0 ? (kj + 1 < g.ny) : 0);
            double a[B2], u[B2], l[B2], uk[B2], p[B2];
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                a[e] = (double)A[(size_t)qk * B2 + e];
                u[e] = (double)lu[(size_t)qdk * B2 + e];
                uk[e] = (double)A[(size_t)qki * B2 + e];
            }
            block_mul<NB>(a, u, l);
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                lu[(size_t)qk * B2 + e] = (LT)l[e];
                if (lo) lo[rec_at(pl, dir * B2 + e, W)] = (LT)l[e];
            }
            block_mul<NB>(l, uk, p);
#pragma unroll
            for (int e = 0; e < B2; ++e) d[e] -= p[e];
            // shared well columns: A_iw -= L_ik U_kw (row k's well blocks
            // follow its 7-point part)
            if (qw0 < q1) {
                const int nupk = (ki + 1 < g.nx) + (kj + 1 < g.ny) + (kk + 1 < g.nz);
                const int qkw0 = qdk + 1 + nupk, qk1 = sys.rowptr[rk + 1];
                for (int q = qw0; q < q1; ++q) {
                    const int col = sys.colind[q];
                    if (T.rtile[col] != tile) continue;
                    for (int qq = qkw0; qq < qk1; ++qq) {
                        if (sys.colind[qq] != col) continue;
                        double ukw[B2], pw[B2];
#pragma unroll
                        for (int e = 0; e < B2; ++e) ukw[e] = (double)lu[(size_t)qq * B2 + e];
                        block_mul<NB>(l, ukw, pw);
#pragma unroll
                        for (int e = 0; e < B2; ++e)
                            lu[(size_t)q * B2 + e] = (LT)((double)lu[(size_t)q * B2 + e] - pw[e]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < B2; ++e) lu[(size_t)qk * B2 + e] = (LT)A[(size_t)qk * B2 + e];
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
    for (int e = 0; e < B2; ++e) {
        lu[(size_t)qd * B2 + e] = (LT)inv[e];
        if (up) up[rec_at(pu, e, W)] = (LT)inv[e];
    }
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

// Sweep records of a tile whose pencils fit the workgroup.  The thread of
// pencil (li, lj) meets cell (li, lj, lk) at step s = li + lj + lk of both
// sweeps; the cell's records hold the blocks it uses there.  Lower records:
// the -z, -y, -x blocks; upper records: the inverted diagonal, then the +x,
// +y, +z blocks; a neighbour outside the tile has a zero block, so the
// sweeps multiply without a branch.  Couplings to wells stay in A's layout.
// The cells of a step are numbered consecutively (ilu_rank_table) and the
// step's records stored in 16-byte chunks of w = 16 / element-size
// elements, chunk by chunk: element j of the cell at position q of step s
// (c cells, first cell number f, ne elements per record rounded up to a
// multiple of w) sits at f * ne + (j / w) * w * c + q * w + j % w, so the
// threads active at one step read and write adjacent chunks.

// Byte offset (from the factors' start) of tile b's lower (upper = false)
// or upper records; a tile's records of one kind take prec * rec_elems
// elements.
__host__ __device__ inline size_t rec_region(const IluTiles &T, int nb, int esize, int b,
                                             bool upper) {
    const size_t lo = (size_t)T.prec * rec_elems(3, nb, esize) * esize;
    const size_t up = (size_t)T.prec * rec_elems(4, nb, esize) * esize;
    const size_t ntiles = (size_t)T.ntx * T.nty * T.ntz;
    size_t off = (size_t)T.poff * esize;
    if (upper) off += ntiles * lo + (size_t)b * up;
    else off += (size_t)b * lo;
    return off;
}

size_t ilu_factor_elems(int nb, long nnzb, const IluTiles &T, int esize) {
    const size_t base = (size_t)nnzb * nb * nb;
    if (T.poff < 0) return base;
    return (size_t)T.poff + (size_t)T.ntx * T.nty * T.ntz * T.prec *
                                (rec_elems(3, nb, esize) + rec_elems(4, nb, esize));
}

__host__ __device__ int ilu_rank_ints(const IluTiles &T) { return T.psteps * T.ty + 2 * T.psteps; }

// Numbering of a tile's cells: step by step (s = li + lj + lk), and within
// a step by (lj, li).  roff[s * T.ty + lj] + li is the number of cell
// (li, lj, s - li - lj); cnt[s] and first[s] are the number of cells of
// step s and the number of its first cell.  Built by the whole workgroup
// (two barriers).
__device__ void ilu_rank_table(const TileBox &tb, const IluTiles &T, int *roff) {
    int *cnt = roff + T.psteps * T.ty, *first = cnt + T.psteps;
    const int S = tb.txe + tb.tye + tb.tze - 2;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        int acc = 0;
        for (int lj = 0; lj < tb.tye; ++lj) {
            const int lo = max(0, s - lj - (tb.tze - 1)), hi = min(tb.txe - 1, s - lj);
            roff[s * T.ty + lj] = acc - lo;
            acc += max(0, hi - lo + 1);
        }
        cnt[s] = acc;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        int base = 0;
        for (int q = 0; q < s; ++q) base += cnt[q];
        for (int lj = 0; lj < tb.tye; ++lj) roff[s * T.ty + lj] += base;
        first[s] = base;
    }
    __syncthreads();
}

// 16 bytes (two doubles or four floats of a block row-major) to raw buffer
// rs at byte offset off, from v[0..16/sizeof(LT))
template <class LT>
__device__ inline void buf_st16(__amdgpu_buffer_rsrc_t rs, int off, const double *v) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(LT) == 8) {
        const double w[2] = {v[0], v[1]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), rs, off, 0, 0);
    } else {
        const float w[4] = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), rs, off, 0, 0);
    }
}

// The hyperplane walk of a tile with sweep records and 2x2 blocks, one
// pencil per thread: the arithmetic of factor_cell_row, row by row in the
// same order, with the inverted pivot and the +x / +y blocks of each
// finished row handed to the threads of the next hyperplane through LDS
// (the -z ones stay in the thread's registers) and the A blocks of a
// thread's next row loaded one step ahead.  Every lane runs every step, on
// its nearest row when it has none at that step, with its loads and stores
// then at the end of raw buffers (zeros, dropped), so no branch separates a
// load from its use.  Tiles with wells of their own order global memory
// between steps (their rows' well columns are updated from the finished rows
// below them).
template <class LT>
__device__ void factor_pencils(const Grid &g, const IluTiles &T, const TileBox &tb, int b,
                               const Sys &sys, LT *lu, long nnzb, int *bad, const int *roff,
                               int *qrow, double *xch, bool wells) {
    constexpr int NB = 2, B2 = 4, ES = sizeof(LT), W = 16 / ES;
    constexpr int kEL = rec_elems(3, NB, ES), kEU = rec_elems(4, NB, ES);
    const int nt = blockDim.x, tid = threadIdx.x;
    const int sxy = tb.txe * tb.tye, ncell = sxy * tb.tze;
    const bool own = tid < sxy;
    const int li = own ? tid % tb.txe : 0, lj = own ? tid / tb.txe : 0;
    const int i = tb.i0 + li, j = tb.j0 + lj;
    const int s0 = li + lj, s1 = s0 + tb.tze - 1, nlev = tb.txe + tb.tye + tb.tze - 2;
    int *qend = qrow + T.prec;
    for (int l = tid; l < ncell; l += nt) {
        const int a = l % tb.txe, c = (l / tb.txe) % tb.tye, e = l / sxy;
        const int r = (tb.i0 + a) + g.nx * ((tb.j0 + c) + g.ny * (tb.k0 + e));
        qrow[l] = sys.rowptr[r];
        qend[l] = sys.rowptr[r + 1];
    }
    __syncthreads();
    const unsigned abytes = (unsigned)((size_t)nnzb * B2 * sizeof(double));
    const unsigned lbytes = (unsigned)((size_t)nnzb * B2 * ES);
    const unsigned lobytes = (unsigned)(T.prec * kEL * ES), upbytes = (unsigned)(T.prec * kEU * ES);
    char *base = reinterpret_cast<char *>(lu);
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(sys.val, abytes);
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(lu, lbytes);
    const __amdgpu_buffer_rsrc_t rlo = make_rsrc(base + rec_region(T, NB, ES, b, false), lobytes);
    const __amdgpu_buffer_rsrc_t rup = make_rsrc(base + rec_region(T, NB, ES, b, true), upbytes);
    auto mine = [&](int s) { return own && s >= s0 && s <= s1; };
    auto clampstep = [&](int s) { return s < s0 ? s0 : (s > s1 ? s1 : s); };
    // the 7-point blocks of a row: -z, -y, -x, diagonal, +x, +y, +z
    struct Row {
        int q[7];
        bool ex[7];
    };
    auto row_at = [&](int s) {
        const int lk = clampstep(s) - s0, k = tb.k0 + lk;
        Row R;
        const int q0 = qrow[li + tb.txe * (lj + tb.tye * lk)];
        R.ex[0] = k > 0; R.ex[1] = j > 0; R.ex[2] = i > 0; R.ex[3] = true;
        R.ex[4] = i + 1 < g.nx; R.ex[5] = j + 1 < g.ny; R.ex[6] = k + 1 < g.nz;
        R.q[0] = q0;
        R.q[1] = R.q[0] + R.ex[0];
        R.q[2] = R.q[1] + R.ex[1];
        R.q[3] = R.q[2] + R.ex[2];
        R.q[4] = R.q[3] + 1;
        R.q[5] = R.q[4] + R.ex[4];
        R.q[6] = R.q[5] + R.ex[5];
        return R;
    };
    // A's blocks m0 .. m0+nm-1 of the row at step s (zeros for a missing
    // block or step)
    auto loadA = [&](int s, int m0, int nm, double (*X)[B2]) {
        const Row R = row_at(s);
        const bool on = mine(s);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= nm) break;
            const int off = (on && R.ex[m0 + m]) ? R.q[m0 + m] * (B2 * 8) : (int)abytes;
#pragma unroll
            for (int e = 0; e < B2; ++e) X[m][e] = buf_ld(ra, off + 8 * e);
        }
    };
    double pz_inv[B2] = {}, pz_u[B2] = {};        // the -z row: inverted pivot, +z block
    auto step = [&](int s, const double (&X)[4][B2]) {
        const bool on = mine(s);
        // the upper blocks, needed only at the end of the step
        double U[3][B2];
        loadA(s, 4, 3, U);
        const int lk = clampstep(s) - s0, k = tb.k0 + lk;
        const int l = li + tb.txe * (lj + tb.tye * lk);
        const Row R = row_at(s);
        const bool in[3] = {lk > 0, lj > 0, li > 0};
        const double *nby = xch + ((size_t)(((s - 1) & 1) * nt + (own && lj > 0 ? tid - tb.txe : tid))) * 3 * B2;
        const double *nbx = xch + ((size_t)(((s - 1) & 1) * nt + (own && li > 0 ? tid - 1 : tid))) * 3 * B2;
        double d[B2], L[3][B2];
#pragma unroll
        for (int e = 0; e < B2; ++e) d[e] = X[3][e];
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            double u[B2], uk[B2];
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                u[e] = dir == 0 ? pz_inv[e] : (dir == 1 ? nby[e] : nbx[e]);
                uk[e] = dir == 0 ? pz_u[e] : (dir == 1 ? nby[2 * B2 + e] : nbx[B2 + e]);
            }
            double l2[B2], p[B2];
            block_mul<NB>(X[dir], u, l2);
            block_mul<NB>(l2, uk, p);
#pragma unroll
            for (int e = 0; e < B2; ++e) {
                L[dir][e] = in[dir] ? l2[e] : 0.0;
                d[e] -= in[dir] ? p[e] : 0.0;
            }
        }
        // well columns of a perforated row (tiles with wells of their own)
        const int qw0 = R.q[6] + R.ex[6];
        const int q1 = on ? qend[l] : qw0;
        for (int q = qw0; q < q1; ++q) {
            const int col = sys.colind[q];
            double acc[B2];
#pragma unroll
            for (int e = 0; e < B2; ++e) acc[e] = (double)(LT)sys.val[(size_t)q * B2 + e];
            if (T.rtile[col] == b)
#pragma unroll
                for (int dir = 0; dir < 3; ++dir) {
                    if (!in[dir]) continue;
                    const int rk = (i - (dir == 2)) + g.nx * ((j - (dir == 1)) + g.ny * (k - (dir == 0)));
                    for (int qq = sys.rowptr[rk]; qq < sys.rowptr[rk + 1]; ++qq) {
                        if (sys.colind[qq] != col) continue;
                        double ukw[B2], pw[B2];
#pragma unroll
                        for (int e = 0; e < B2; ++e) ukw[e] = (double)lu[(size_t)qq * B2 + e];
                        block_mul<NB>(L[dir], ukw, pw);
#pragma unroll
                        for (int e = 0; e < B2; ++e) acc[e] = (double)(LT)(acc[e] - pw[e]);
                    }
                }
#pragma unroll
            for (int e = 0; e < B2; ++e) lu[(size_t)q * B2 + e] = (LT)acc[e];
        }
        double inv[B2];
        if (!invert_block<NB>(d, inv)) {
            if (on) *bad = 1;
#pragma unroll
            for (int e = 0; e < B2; ++e) inv[e] = (e % (NB + 1) == 0) ? 1.0 : 0.0;
        }
        // the row in lu: L (A's block for a neighbour outside the tile), the
        // inverted pivot, A's upper blocks
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int off = (on && R.ex[m]) ? R.q[m] * (B2 * ES) : (int)lbytes;
#pragma unroll
            for (int c = 0; c < B2 / W; ++c) {
                double v[W];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const int e = c * W + w;
                    v[w] = m < 3 ? (in[m] ? L[m][e] : X[m][e]) : (m == 3 ? inv[e] : U[m - 4][e]);
                }
                buf_st16<LT>(rl, off + 16 * c, v);
            }
        }
        // the sweep records (zero blocks towards neighbours outside the tile)
        const bool hin[3] = {li + 1 < tb.txe, lj + 1 < tb.tye, lk + 1 < tb.tze};
        const int sc = clampstep(s);
        const RecPos pl = rec_pos(T, roff, sc, li, lj, kEL, W), pu = rec_pos(T, roff, sc, li, lj, kEU, W);
#pragma unroll
        for (int c = 0; c < kEL / W; ++c) {
            double v[W];
#pragma unroll
            for (int w = 0; w < W; ++w) v[w] = L[(c * W + w) / B2][(c * W + w) % B2];
            buf_st16<LT>(rlo, on ? (pl.start + c * pl.stride) * ES : (int)lobytes, v);
        }
#pragma unroll
        for (int c = 0; c < kEU / W; ++c) {
            double v[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int m = (c * W + w) / B2, e = (c * W + w) % B2;
                v[w] = m == 0 ? inv[e] : (hin[m - 1] ? U[m - 1][e] : 0.0);
            }
            buf_st16<LT>(rup, on ? (pu.start + c * pu.stride) * ES : (int)upbytes, v);
        }
        // for the next hyperplane: this row's inverted pivot (as stored) and
        // its +x, +y blocks in LDS, its +z block and pivot in registers
        double *mine_slot = xch + ((size_t)((s & 1) * nt + tid)) * 3 * B2;
#pragma unroll
        for (int e = 0; e < B2; ++e) {
            const double is = (double)(LT)inv[e];
            mine_slot[e] = is;
            mine_slot[B2 + e] = U[0][e];
            mine_slot[2 * B2 + e] = U[1][e];
            pz_inv[e] = is;
            pz_u[e] = U[2][e];
        }
    };
    double XA[4][B2], XB[4][B2];                 // lower and diagonal blocks, a step ahead
    loadA(0, 0, 4, XA);
    for (int s = 0; s < nlev; s += 2) {
        loadA(s + 1, 0, 4, XB);
        step(s, XA);
        if (wells) __syncthreads();
        else lds_barrier();
        loadA(s + 2, 0, 4, XA);
        step(s + 1, XB);
        if (wells) __syncthreads();
        else lds_barrier();
    }
}

// One workgroup per tile, then one for the wells that stand alone.  The
// tile's well rows are copied from A first; its cell rows are read from A
// as they are factored, hyperplane by hyperplane, and tiles with sweep
// records write each cell's as soon as its row is done.
template <int NB, class LT>
__device__ __forceinline__ void ilu_factor_body(int hb, int nblk, const Grid &g, const IluTiles &T,
                                                const Sys &sys, LT *lu, int *bad) {
    constexpr int B2 = NB * NB;
    const int b = xcd_block(hb, nblk);                // contiguous tiles per XCD
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
    extern __shared__ double fsm[];
    double *xch = fsm;                                   // pencil path: 2 x threads x 3 blocks
    int *roff = reinterpret_cast<int *>(fsm + (NB == 2 ? (size_t)2 * blockDim.x * 3 * B2 : 0));
    if (T.poff >= 0) ilu_rank_table(tb, T, roff);
    // the tile's well rows are factored in place after its cells (the cell
    // rows are read from A as they are factored)
    for (int e = T.twp[b]; e < T.twp[b + 1]; ++e) {
        const int r = g.n + T.tw[e];
        copy_blocks(sys.val, lu, sys.rowptr[r], sys.rowptr[r + 1], B2);
    }
    __syncthreads();
    if constexpr (NB == 2) {
        if (T.poff >= 0) {
            factor_pencils<LT>(g, T, tb, b, sys, lu, T.nnzb, bad, roff, roff + ilu_rank_ints(T), xch,
                               T.twp[b + 1] > T.twp[b]);
            __syncthreads();
            for (int e = T.twp[b] + threadIdx.x; e < T.twp[b + 1]; e += blockDim.x)
                factor_row<NB, LT>(g.n + T.tw[e], T, sys, lu, bad);
            return;
        }
    }
    // other tiles: the cell rows copied first (each x-row of the tile one
    // contiguous run of blocks), then factored in place from the copy
    for (int seg = 0; seg < tb.tye * tb.tze; ++seg) {
        const int j = tb.j0 + seg % tb.tye, k = tb.k0 + seg / tb.tye;
        const int r0 = tb.i0 + g.nx * (j + g.ny * k);
        copy_blocks(sys.val, lu, sys.rowptr[r0], sys.rowptr[r0 + tb.txe], B2);
    }
    __syncthreads();
    const int nlev = tb.txe + tb.tye + tb.tze - 2;
    for (int s = 0; s < nlev; ++s) {
        for (int p = threadIdx.x; p < tb.txe * tb.tye; p += blockDim.x) {
            const int li = p % tb.txe, lj = p / tb.txe, lk = s - li - lj;
            if (lk < 0 || lk >= tb.tze) continue;
            const int i = tb.i0 + li, j = tb.j0 + lj, k = tb.k0 + lk;
            LT *lo = nullptr, *up = nullptr;
            RecPos pl{}, pu{};
            if (T.poff >= 0) {
                constexpr int W = 16 / sizeof(LT);
                pl = rec_pos(T, roff, s, li, lj, rec_elems(3, NB, sizeof(LT)), W);
                pu = rec_pos(T, roff, s, li, lj, rec_elems(4, NB, sizeof(LT)), W);
                char *base = reinterpret_cast<char *>(lu);
                lo = reinterpret_cast<LT *>(base + rec_region(T, NB, sizeof(LT), b, false));
                up = reinterpret_cast<LT *>(base + rec_region(T, NB, sizeof(LT), b, true));
            }
            factor_cell_row<NB, LT, LT>(i, j, k, g, T, tb, b, sys, lu, lu, bad, lo, up, pl, pu);
        }
        __syncthreads();
    }
    for (int e = T.twp[b] + threadIdx.x; e < T.twp[b + 1]; e += blockDim.x)
        factor_row<NB, LT>(g.n + T.tw[e], T, sys, lu, bad);
}

template <int NB, class LT>
__global__ __launch_bounds__(256) void k_ilu_factor(Grid g, IluTiles T, Sys sys, LT *lu,
                                                    int *bad) {
    ilu_factor_body<NB, LT>(blockIdx.x, gridDim.x, g, T, sys, lu, bad);
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
                               int q0 = -1, int q1 = -1) {
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = (double)R.b[(size_t)r * NB + u];
    if (!R.ap) return;
    if (q0 < 0) q0 = sys.rowptr[r];
    if (q1 < 0) q1 = sys.rowptr[r + 1];
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

// The right sides of H cell rows of the grid's 7-point pattern (cells
// (ci, cj, ck), rows rr, blocks q0 .. q1 - 1): rhs_row's values, summed in
// the same order.  A cell row holds the blocks of its existing neighbours
// first, in column order (-z, -y, -x, the cell, +x, +y, +z), then its well
// columns.  A neighbour's level-0 entry follows from the cell's own (the
// colour flips, the unsplit index moves by the neighbour's offset), so only
// well columns read colsplit.  Every row's stencil loads are issued before
// the first product: a missing neighbour loads a block of the row, reads
// its entry past the end of a raw buffer (zero, without a memory access)
// and is dropped by a select.
template <int NB, int H, class RT>
__device__ inline void rhs_cells(const RT &R, const Grid &g, const int (&ci)[H],
                                 const int (&cj)[H], const int (&ck)[H], const int (&rr)[H],
                                 const int (&q0)[H], const int (&q1)[H], double (&acc)[H][NB]) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[h][u] = (double)R.b[(size_t)rr[h] * NB + u];
    if (!R.ap) return;
    const int half = R.nsplit >> 1, pz = R.nxp * g.ny;
    const int dcc[7] = {-pz, -R.nxp, -1, 0, 1, R.nxp, pz};
    const __amdgpu_buffer_rsrc_t rpx = make_rsrc(R.px, (unsigned)R.nsplit * 8u);
    bool ex[H][7];
    double a[H][7][NB], p[H][7];
    int qe[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int i = ci[h], j = cj[h], k = ck[h];
        const bool e[7] = {k > 0, j > 0, i > 0, true, i + 1 < g.nx, j + 1 < g.ny, k + 1 < g.nz};
        const int cc = i + R.nxp * (j + g.ny * k);
        const int par = (i + j + k) & 1;
        const int own = (par ? half : 0) + (cc >> 1), oth = par ? 0 : half;
        int q = q0[h];
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            ex[h][d] = e[d];
            const int qd = min(q, q1[h] - 1);
            q += e[d];
            const int sd = d == 3 ? own : oth + ((cc + dcc[d]) >> 1);
#pragma unroll
            for (int u = 0; u < NB; ++u) a[h][d][u] = (double)R.ap[(size_t)qd * NB + u];
            p[h][d] = buf_ld(rpx, e[d] ? sd * 8 : R.nsplit * 8);
        }
        qe[h] = q;
    }
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int d = 0; d < 7; ++d)
#pragma unroll
            for (int u = 0; u < NB; ++u)
                acc[h][u] -= (ex[h][d] ? a[h][d][u] : 0.0) * (ex[h][d] ? p[h][d] : 0.0);
#pragma unroll
    for (int h = 0; h < H; ++h)
        for (int q = qe[h]; q < q1[h]; ++q) {
            const double pq = R.px[R.colsplit[q]];
#pragma unroll
            for (int u = 0; u < NB; ++u) acc[h][u] -= (double)R.ap[(size_t)q * NB + u] * pq;
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

// The NBLK blocks of a sweep record: 16-byte chunk c at byte offset
// off + c * stride of buffer rs (an offset past the buffer's end gives
// zeros, without a memory access).
template <int NB, class LT, int NBLK>
__device__ inline void load_rec(Blk<NB> (&X)[NBLK], __amdgpu_buffer_rsrc_t rs, int off, int stride) {
    constexpr int B2 = NB * NB, W = 16 / sizeof(LT), nc = rec_elems(NBLK, NB, sizeof(LT)) / W;
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 raw[nc];
#pragma unroll
    for (int c = 0; c < nc; ++c) raw[c] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + c * stride, 0, 0);
    LT e[nc * W];
    __builtin_memcpy(e, raw, sizeof(raw));
#pragma unroll
    for (int m = 0; m < NBLK; ++m)
#pragma unroll
        for (int q = 0; q < B2; ++q) X[m].v[q] = (double)e[m * B2 + q];
}

// Both sweeps over the cells of a tile whose (li, lj) pencils fit the
// workgroup: thread (li, lj) owns the pencil and meets its cells in order
// of lk, one per hyperplane, reading their blocks from the tile's sweep
// records two steps ahead.  Row starts and the right side are staged in LDS
// first.  Same arithmetic, same order, as the general sweeps.
template <int NB, class LT, class RT>
__device__ void solve_cells_pencils(const Grid &g, const TileBox &tb, const Sys &sys,
                                    const LT *__restrict__ lu, const RT &R,
                                    double *y, int *rp, const IluTiles &T, int blk, int w0, int nwt,
                                    int ncell) {
    constexpr int B2 = NB * NB;
    const int sxy = tb.txe * tb.tye;
    int *re = rp + ncell;                          // row ends
    int *roff = re + ncell;                        // record order
    ilu_rank_table(tb, T, roff);
    // kH rows per thread at a time so their loads overlap (a slot past the
    // tile's cells works on its last cell and stores nothing: no branch
    // between the loads)
    constexpr int kH = NB == 2 ? 3 : 2;
    for (int l0 = threadIdx.x; l0 < ncell; l0 += kH * blockDim.x) {
        int rr[kH], q0[kH], q1[kH], ci[kH], cj[kH], ck[kH];
#pragma unroll
        for (int h = 0; h < kH; ++h) {
            const int l = min(l0 + h * (int)blockDim.x, ncell - 1);
            ci[h] = tb.i0 + l % tb.txe;
            cj[h] = tb.j0 + (l / tb.txe) % tb.tye;
            ck[h] = tb.k0 + l / sxy;
            rr[h] = ci[h] + g.nx * (cj[h] + g.ny * ck[h]);
            q0[h] = sys.rowptr[rr[h]];
            q1[h] = sys.rowptr[rr[h] + 1];
        }
        double acc[kH][NB];
        rhs_cells<NB, kH>(R, g, ci, cj, ck, rr, q0, q1, acc);
#pragma unroll
        for (int h = 0; h < kH; ++h)
            if (l0 + h * (int)blockDim.x < ncell) {
                const int l = l0 + h * blockDim.x;
                rp[l] = q0[h];
                re[l] = q1[h];
#pragma unroll
                for (int u = 0; u < NB; ++u) y[(size_t)l * NB + u] = acc[h][u];
            }
    }
    __syncthreads();
    const bool own = (int)threadIdx.x < sxy;
    const int li = own ? threadIdx.x % tb.txe : 0, lj = own ? threadIdx.x / tb.txe : 0;
    const int i = tb.i0 + li, j = tb.j0 + lj;
    const int nlev = tb.txe + tb.tye + tb.tze - 2;
    // the thread's cells come at steps s0 .. s1; a prefetch for a step
    // outside them reads past the end of the tile's record buffer, which
    // returns zeros without a memory access, so every lane issues the same
    // loads and no wait covers more than the record about to be used
    const int s0 = li + lj, s1 = s0 + tb.tze - 1;
    auto mine = [&](int s) { return own && s >= s0 && s <= s1; };
    // a lane without a pencil (tiles narrower than the workgroup) reads and
    // writes a slot of its own past the tile's vector, never a cell's
    const int ldummy = ncell + T.maxwells;
    auto clampstep = [&](int s) { return s < s0 ? s0 : (s > s1 ? s1 : s); };
    // forward: y -= Lz y(-z) + Ly y(-y) + Lx y(-x), zero blocks at the tile's
    // faces (the cell's own y stands in for the missing neighbour)
    Blk<NB> fa[3], fb[3];
    const char *lub = reinterpret_cast<const char *>(lu);
    constexpr int kES = sizeof(LT), kW = 16 / kES;
    constexpr int kEL = rec_elems(3, NB, kES), kEU = rec_elems(4, NB, kES);
    const int nrec = T.prec;
    // byte offset and chunk stride of the record of step s (for a step
    // without a cell of this thread: the end of the buffer, which reads
    // zeros)
    auto recoff = [&](int s, int ne, int &stride) {
        const RecPos p = rec_pos(T, roff, clampstep(s), li, lj, ne, kW);
        stride = p.stride * kES;
        return mine(s) ? p.start * kES : nrec * ne * kES;
    };
    const __amdgpu_buffer_rsrc_t rsl = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char *>(lub + rec_region(T, NB, sizeof(LT), blk, false)), 0, nrec * kEL * kES,
        kBufferWord3);
    auto lower = [&](int s, Blk<NB> (&X)[3]) {
        int stride;
        const int off = recoff(s, kEL, stride);
        load_rec<NB, LT, 3>(X, rsl, off, stride);
    };
    // every lane computes (a lane without a cell at step s on its nearest
    // cell, discarded), so the record buffers are consumed on one path
    auto fstep = [&](int s, const Blk<NB> (&X)[3]) {
        const int lk = clampstep(s) - s0, l = own ? li + tb.txe * (lj + tb.tye * lk) : ldummy;
        double acc[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] = y[(size_t)l * NB + u];
        sub_mv<NB>(acc, X[0].v, y + (size_t)(own && lk > 0 ? l - sxy : l) * NB);
        sub_mv<NB>(acc, X[1].v, y + (size_t)(own && lj > 0 ? l - tb.txe : l) * NB);
        sub_mv<NB>(acc, X[2].v, y + (size_t)(own && li > 0 ? l - 1 : l) * NB);
        // a lane without a cell at step s writes back its own cell's value
        // unchanged (pencils are disjoint, so no other lane writes there)
        const bool on = mine(s);
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double old = y[(size_t)l * NB + u];
            y[(size_t)l * NB + u] = on ? acc[u] : old;
        }
    };
    // two record buffers by the parity of the step: the one used at step s
    // is refilled for step s + 2 right after (an even number of steps, the
    // last one possibly empty, keeps the loop body free of branches)
    lower(0, fa);
    __builtin_amdgcn_sched_barrier(0);            // keep the loads in step order
    lower(1, fb);
    for (int s = 0; s < nlev; s += 2) {
        fstep(s, fa);
        lower(s + 2, fa);
        lds_barrier();
        fstep(s + 1, fb);
        lower(s + 3, fb);
        lds_barrier();
    }
    __syncthreads();
    solve_tile_wells<NB, LT>(g, tb, sys, lu, R, y, T, w0, nwt, ncell);
    __syncthreads();
    // backward: y -= Ux y(+x) + Uy y(+y) + Uz y(+z) + the tile's wells, then
    // x = -inv(U_kk) y (the diagonal record holds the inverted pivot)
    Blk<NB> ga[4], gb[4];
    const __amdgpu_buffer_rsrc_t rsu = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char *>(lub + rec_region(T, NB, sizeof(LT), blk, true)), 0, nrec * kEU * kES,
        kBufferWord3);
    auto upper = [&](int s, Blk<NB> (&X)[4]) {
        int stride;
        const int off = recoff(s, kEU, stride);
        load_rec<NB, LT, 4>(X, rsu, off, stride);
    };
    auto bstep = [&](int s, const Blk<NB> (&X)[4]) {
        const bool on = mine(s);
        const int lk = clampstep(s) - s0, k = tb.k0 + lk;
        const int l = own ? li + tb.txe * (lj + tb.tye * lk) : ldummy;
        double acc[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] = y[(size_t)l * NB + u];
        sub_mv<NB>(acc, X[1].v, y + (size_t)(own && li + 1 < tb.txe ? l + 1 : l) * NB);
        sub_mv<NB>(acc, X[2].v, y + (size_t)(own && lj + 1 < tb.tye ? l + tb.txe : l) * NB);
        sub_mv<NB>(acc, X[3].v, y + (size_t)(own && lk + 1 < tb.tze ? l + sxy : l) * NB);
        // well columns (perforated cells): the wells of this tile (none to
        // look for in a tile without wells of its own, the common case: the
        // loads of the loop would stall the step)
        const int qw = rp[own ? l : 0] + (k > 0) + (j > 0) + (i > 0) + 1 + (i + 1 < g.nx) + (j + 1 < g.ny) +
                       (k + 1 < g.nz);
        const int qe = on && nwt > 0 ? re[own ? l : 0] : qw;
        for (int q = qw; q < qe; ++q) {
            const int w = sys.colind[q] - g.n;
            if (T.rtile[g.n + w] == blk)
                sub_mv<NB>(acc, lu + (size_t)q * B2, y + (size_t)(ncell + T.wlocal[w]) * NB);
        }
        double xr[NB] = {};
        sub_mv<NB>(xr, X[0].v, acc);
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double old = y[(size_t)l * NB + u];
            y[(size_t)l * NB + u] = on ? -xr[u] : old;
        }
    };
    upper(nlev - 1, ga);
    __builtin_amdgcn_sched_barrier(0);
    upper(nlev - 2, gb);
    for (int s = nlev - 1; s >= 0; s -= 2) {
        bstep(s, ga);
        upper(s - 2, ga);
        lds_barrier();
        bstep(s - 1, gb);
        upper(s - 3, gb);
        lds_barrier();
    }
}

// x = M^-1 rhs: forward (L y = rhs, L unit lower) and backward (U x = y)
// inside every tile; for the CPR second stage the first-stage correction is
// added to the first slot of every row of x.
template <int NB, class LT, class VT>
__device__ __forceinline__ void ilu_solve_body(int hb, int nblk, const Grid &g, const IluTiles &T,
                                               const Sys &sys, const LT *__restrict__ lu,
                                               const IluRhs<VT, LT> &R, VT *__restrict__ x,
                                               double *y) {
    constexpr int B2 = NB * NB;
    // each XCD takes one contiguous run of tiles (neighbouring tiles share
    // lines of the level-0 iterate and of the rows at their faces)
    const int blk = xcd_block(hb, nblk);
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
    if (T.poff >= 0 && sxy <= (int)blockDim.x) {
        solve_cells_pencils<NB, LT>(g, tb, sys, lu, R, y, reinterpret_cast<int *>(y + (size_t)(ncell + T.maxwells + 1) * NB),
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
    // x = y + the first-stage correction, kW rows per thread at a time with
    // their corrections' loads issued together (a cell's level-0 entry from
    // its coordinates, as in rhs_cells; a slot past the tile's rows repeats
    // its last row and stores nothing)
    constexpr int kW = 4;
    const int nrow = ncell + nwt;
    for (int l0 = threadIdx.x; l0 < nrow; l0 += kW * blockDim.x) {
        int rr[kW], ll[kW];
        double mu[kW];
#pragma unroll
        for (int h = 0; h < kW; ++h) {
            const int l = min(l0 + h * (int)blockDim.x, nrow - 1);
            ll[h] = l;
            int sp;
            if (l < ncell) {
                const int li = l % tb.txe, lj = (l / tb.txe) % tb.tye, lk = l / sxy;
                const int i = tb.i0 + li, j = tb.j0 + lj, k = tb.k0 + lk;
                rr[h] = i + g.nx * (j + g.ny * k);
                sp = (((i + j + k) & 1) ? (R.nsplit >> 1) : 0) + ((i + R.nxp * (j + g.ny * k)) >> 1);
            } else {
                const int w = T.tw[w0 + (l - ncell)];
                rr[h] = n + w;
                sp = R.nsplit + w;
            }
            mu[h] = R.ap ? R.px[sp] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < kW; ++h) {
            if (l0 + h * (int)blockDim.x >= nrow) continue;
            const int r = rr[h], l = ll[h];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                double c = 0.0;
                if (R.ap) c = (R.pw && r < n) ? R.pw[(size_t)r * NB + u] * mu[h] : (u == 0 ? mu[h] : 0.0);
                x[(size_t)r * NB + u] = (VT)(y[(size_t)l * NB + u] + c);
            }
        }
    }
}

template <int NB, class LT, class VT>
__global__ __launch_bounds__(256) void k_ilu_solve(Grid g, IluTiles T, Sys sys,
                                                   const LT *__restrict__ lu, IluRhs<VT, LT> R,
                                                   VT *__restrict__ x) {
    extern __shared__ double y[];
    ilu_solve_body<NB, LT, VT>(blockIdx.x, gridDim.x, g, T, sys, lu, R, x, y);
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
    const size_t lds = ilu_factor_lds(nb, T);
    if (nb == 2)
        hipLaunchKernelGGL((k_ilu_factor<2, LT>), dim3(nblk), dim3(bs), lds, s, g, T, sys, lu, bad);
    else
        hipLaunchKernelGGL((k_ilu_factor<3, LT>), dim3(nblk), dim3(bs), lds, s, g, T, sys, lu, bad);
}

void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, double *lu,
                       int *bad) {
    ilu_factor_impl(s, nb, g, T, sys, lu, bad);
}

void launch_ilu_factor(hipStream_t s, int nb, Grid g, const IluTiles &T, Sys sys, float *lu,
                       int *bad) {
    ilu_factor_impl(s, nb, g, T, sys, lu, bad);
}

// LDS of the factorisation: the exchange slots and row starts / ends of the
// pencil path (2x2 blocks), then the record order
size_t ilu_factor_lds(int nb, const IluTiles &T) {
    if (T.poff < 0) return 0;
    const size_t xch = nb == 2 ? (size_t)2 * ilu_threads(T) * 3 * nb * nb * sizeof(double) : 0;
    const size_t rows = nb == 2 ? (size_t)2 * T.prec * sizeof(int) : 0;
    return xch + (size_t)ilu_rank_ints(T) * sizeof(int) + rows;
}

int ilu_threads(const IluTiles &T) {
    const int pairs = T.tx * T.ty;
    return pairs >= 256 ? 256 : ((pairs + 63) / 64) * 64;
}

size_t ilu_solve_lds(int nb, const IluTiles &T) {
    // the tile's vector and a spare slot, then its row starts and ends and
    // its record order (pencil sweeps)
    return (size_t)(T.tx * T.ty * T.tz + T.maxwells + 1) * nb * sizeof(double) +
           (size_t)2 * T.tx * T.ty * T.tz * sizeof(int) +
           (T.poff >= 0 ? (size_t)ilu_rank_ints(T) * sizeof(int) : 0);
}

template <class LT, class VT>
static hipError_t allow_lds_impl(int nb, size_t bytes) {
    hipError_t e;
    if (nb == 2) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_solve<2, LT, VT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_factor<2, LT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        return e;
    }
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_solve<3, LT, VT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ilu_factor<3, LT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
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

// ---------------------------------------------------------------------------
// batched launches over the members of an ensemble (every member's tiles,
// one workgroup each, with the member's CPR right-hand side)

template <int NB>
__global__ __launch_bounds__(256) void kb_ilu_factor(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    ilu_factor_body<NB, double>(b, nb, M.g, M.T, M.sys, M.lu, M.ilu_bad);
}

// z = M^-1 v for the first vector of a restart cycle (j < 0: V_0 -> Z_0) or
// the new Arnoldi vector (j >= 0: V_{j+1} -> Z_{j+1})
template <int NB>
__global__ __launch_bounds__(256) void kb_ilu_solve(const Member *__restrict__ mem, Batch B, int j) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    extern __shared__ double y[];
    const size_t off = (size_t)(j + 1) * M.nvec;
    IluRhs<double, double> R{M.V + off, M.ap, M.colsplit, M.split0, M.lv[0].x, 2 * M.lv[0].half,
                             nullptr};
    R.nxp = M.lv[0].nxp;
    ilu_solve_body<NB, double, double>(b, nb, M.g, M.T, M.sys, M.lu, R, M.Z + off, y);
}

void launchb_ilu_factor(hipStream_t s, int nb, const Member *mem, Batch B, int total, int threads,
                        size_t lds) {
    if (total <= 0) return;
    if (nb == 2)
        hipLaunchKernelGGL(kb_ilu_factor<2>, dim3(total), dim3(threads), lds, s, mem, B);
    else
        hipLaunchKernelGGL(kb_ilu_factor<3>, dim3(total), dim3(threads), lds, s, mem, B);
}

void launchb_ilu_solve(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j,
                       int threads, size_t lds) {
    if (total <= 0) return;
    if (nb == 2)
        hipLaunchKernelGGL(kb_ilu_solve<2>, dim3(total), dim3(threads), lds, s, mem, B, j);
    else
        hipLaunchKernelGGL(kb_ilu_solve<3>, dim3(total), dim3(threads), lds, s, mem, B, j);
}

hipError_t ilu_batch_allow_lds(int nb, size_t bytes) {
    hipError_t e;
    if (nb == 2) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_ilu_solve<2>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_ilu_factor<2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        return e;
    }
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_ilu_solve<3>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_ilu_factor<3>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return e;
}

}  // namespace fim
