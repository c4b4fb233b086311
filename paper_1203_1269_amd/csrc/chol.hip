// Blocked right-looking Cholesky R_delta = L L' in FP64 for a batch of
// matrices (the factorisation the paper uses for the determinant and the
// solves, Sec. 2 and Sec. 3 "CPU implementation"; its GPU code used a
// library LU instead, Sec. 3).
//
// Two-level blocking:
//   outer panels of OUTER_NB = 512 columns (GP_MIXED_RANK = 768 for GP_MIXED,
//   the rank of its INT8 updates); each is factored by inner steps of TB = 64
//   columns, left-looking inside the panel (update of the 64-column block by
//   the panel's earlier blocks, POTRF of its 64 x 64 diagonal tile, TRSM of
//   the rows below it); then the trailing matrix receives one right-looking
//   rank-OUTER_NB update (SYRK/GEMM on FP64 MFMA), which carries most of the
//   n^3/3 flops.  With K = 512 each 128 x 128 output tile does 16.8 MFLOP per
//   256 KiB of C traffic, far above the FP64 ridge of the chip (78.6 TFLOP/s
//   over 8 TB/s); 512 measured 4% faster than 256 and 768 at n = 4096.
#include <math.h>

#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"

namespace gpk {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// Quad broadcast: every lane of each group of 4 lanes receives the value of
// lane Q of its group (DPP quad_perm, no LDS traffic).
template <int Q>
__device__ __forceinline__ double quad_bcast_q(double v)
{
    constexpr int ctrl = Q * 0x55;   // quad_perm [Q, Q, Q, Q]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double quad_bcast(double v, int q)
{
    switch (q & 3) {
    case 0: return quad_bcast_q<0>(v);
    case 1: return quad_bcast_q<1>(v);
    case 2: return quad_bcast_q<2>(v);
    default: return quad_bcast_q<3>(v);
    }
}

// ---------------------------------------------------------------------------
// POTRF of one 64 x 64 diagonal tile per matrix.  Right-looking, column by
// column: L_jj = sqrt(a_jj), L_ij = a_ij / L_jj, then the rank-1 update of the
// columns right of j.  The tile lives in registers: 4 lanes per row, lane q
// of row r holds columns q, q+4, ..., q+60.  Per column one LDS broadcast
// (double-buffered, one barrier).  Division by the pivot is a multiplication
// by its reciprocal.  Also writes 2 sum_j ln L_jj of the tile (wave-level
// reduction) and the first failing pivot (1-based, global) into info.
// With K > 0 the tile first receives its update by the K columns [kc0, c0)
// of the same outer panel (left-looking inside the panel): C - P P^T for the
// tile's rows P of those columns, on FP64 MFMA (wave w: columns 16w..16w+15,
// the 16x16x4 operand layouts of the trailing update below, D[i][j] in lane
// j + 16 (i % 4), element i / 4), staged through LDS.  The accumulators
// start at -C and gather +P P^T: on a diagonal the products shrink the
// running sum towards the small pivot, so each rounding is relative to that
// shrinking sum (summing P P^T from zero and subtracting it from C at the
// end measured 3-4x larger errors on ill-conditioned matrices).

constexpr int PO_THREADS = 256;
#ifndef PT_NSETS
#define PT_NSETS 4   // fragment sets in flight in the in-panel updates
#endif

__global__ __launch_bounds__(PO_THREADS)
void potrf_diag_kernel(double *__restrict__ A0, int lda0, size_t bstride, int c0, int kc0,
                       int K, int32_t *__restrict__ info, double *__restrict__ lpart,
                       int nparts, double *__restrict__ lk0, const uint8_t *__restrict__ mask,
                       const RagMat *__restrict__ rag)
{
    if (mask && !mask[blockIdx.x]) return;   // uniform over the workgroup
    __shared__ double col[2][TB];
    __shared__ double dg[TB];
    __shared__ double ub[TB][TB + 1];   // U of the in-panel update (K > 0)
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int q = tid & 3, r = tid >> 2;
    int lda = lda0;
    size_t boff = (size_t)b * bstride;
    if (rag) {   // ragged batch: this matrix may end before column block c0
        if (c0 >= rag[b].live) return;
        lda = rag[b].lda;
        boff = rag[b].off;
    }
    double *A = A0 + boff + (size_t)c0 + (size_t)c0 * lda;

    if (K > 0) {   // uniform
        const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
        const double *P = A0 + boff + (size_t)c0 + (size_t)(kc0 + g) * lda;
        dbl4 u[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const double *pc = A + (size_t)(16 * rb + g) + (size_t)(16 * wave + li) * lda;
            u[rb] = -(dbl4){pc[0], pc[4], pc[8], pc[12]};
        }
        // PT_NSETS fragment sets in flight (K is a multiple of 64), each
        // reloaded right after its MFMAs; reloads past the end re-read the
        // set just used (in bounds, unused)
        constexpr int NS = PT_NSETS;
        const size_t step4 = (size_t)4 * lda;
        double fa[NS][4], fb[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) fa[st][rb] = P[st * step4 + 16 * rb + li];
            fb[st] = P[st * step4 + 16 * wave + li];
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int k = 0; k < K; k += 4 * NS) {
#pragma unroll
            for (int st = 0; st < NS; ++st) {
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    u[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[st][rb], fb[st], u[rb], 0, 0, 0);
                const size_t nx = (k + 4 * (NS + st) < K) ? (size_t)(NS + st) * step4
                                                          : (size_t)st * step4;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) fa[st][rb] = P[nx + 16 * rb + li];
                fb[st] = P[nx + 16 * wave + li];
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            }
            P += NS * step4;
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            ub[16 * rb + g][16 * wave + li] = -u[rb].x;
            ub[16 * rb + 4 + g][16 * wave + li] = -u[rb].y;
            ub[16 * rb + 8 + g][16 * wave + li] = -u[rb].z;
            ub[16 * rb + 12 + g][16 * wave + li] = -u[rb].w;
        }
        __syncthreads();
    }


    double a[16];
#pragma unroll
    for (int m = 0; m < 16; ++m)
        a[m] = K > 0 ? ub[r][q + 4 * m] : A[(size_t)r + (size_t)(q + 4 * m) * lda];

    int first_bad = 0;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
        const int qj = j & 3, mj = j >> 2;
        double *cb = col[j & 1];
        if (q == qj) cb[r] = a[mj];
        __syncthreads();
        const double piv = cb[j];
        if (!(piv > 0.0) && first_bad == 0) first_bad = c0 + j + 1;
        const double l = sqrt(piv);
        const double linv = 1.0 / l;
        const double lrj = cb[r] * linv;
        if (q == qj) a[mj] = (r == j) ? l : ((r > j) ? lrj : 0.0);
        if (tid == 0) dg[j] = l;
#pragma unroll
        for (int m = mj; m < 16; ++m) {
            const int c = q + 4 * m;
            if (m > mj || q > qj) a[m] = fma(-lrj, cb[c] * linv, a[m]);
        }
    }
    // the factor, and a copy for the TRSM of this step: column-major,
    // strict upper triangle zero, diagonal replaced by 1 / L_jj
    double *lk = lk0 + (size_t)b * TB * TB;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int c = q + 4 * m;
        const double v = (r >= c) ? a[m] : 0.0;
        A[(size_t)r + (size_t)c * lda] = v;
        lk[(size_t)c * TB + r] = (r == c) ? 1.0 / v : v;
    }
    __syncthreads();
    if (tid < TB) {
        double v = log(dg[tid]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (tid == 0) {
            lpart[(size_t)b * nparts + c0 / TB] = 2.0 * v;
            if (first_bad != 0 && info[b] == 0) info[b] = first_bad;
        }
    }
}

// ---------------------------------------------------------------------------
// Rows below the diagonal tile, fused: the in-panel update of the 64-column
// block (left-looking, by the K columns [kc0, c0) of the same outer panel)
// and then the TRSM X L_kk' = A, i.e. per row
// x_j = (a_j - sum_{m<j} x_m L_jm) / L_jj.
// One wave per 16 PT_RB rows, the block held as X^T in 4 x PT_RB
// accumulator tiles of the 16x16x4 FP64 MFMA: tile (cb, rb) holds X^T rows 16 cb .. (columns of
// X) by columns 16 rb .. (rows of X), lane li + 16 g, element e being
// X(row 16 rb + li, column 16 cb + 4 e + g).  In that layout element q of
// every lane is exactly the B operand (B[k][j] in lane j + 16 k) of k-step q
// of a product with X^T on the right, so no data moves between lanes for
// the MFMA parts:
//   update:  X^T -= P_kk P_rows^T   (A operand: rows of the diagonal tile,
//            B operand: the wave's rows, both over the panel columns);
//   TRSM, per 16-column block jb of L_kk: forward substitution inside the
//            block (column by column; the finished column is broadcast from
//            the 16 lanes that hold it, L from LDS), then
//            X^T(cb) -= L(cb, jb) X^T(jb) on MFMA for the later blocks cb.
// No inverse is formed: the arithmetic is that of a blocked forward
// substitution.  L_kk is the copy written by potrf_diag (diagonal holding
// 1 / L_jj), staged in LDS once per workgroup.  Rows come in whole waves
// (the row limit is a multiple of 64).  PT_RB = 2 (32 rows per wave) keeps
// the tile and two fragment sets in the 256 registers of two waves per SIMD.

#ifndef PT_RB
#define PT_RB 2
#endif

constexpr int TR_THREADS = 256;
constexpr int TR_ROWS = 4 * 16 * PT_RB;   // 4 waves

__global__ __launch_bounds__(TR_THREADS, 2)
void panel_trsm_kernel(double *__restrict__ A0, int lda0, size_t bstride, int np, int c0,
                       int kc0, int K, const double *__restrict__ lk0,
                       const uint8_t *__restrict__ mask, const RagMat *__restrict__ rag)
{
    const int b = blockIdx.y;
    if (mask && !mask[b]) return;   // uniform over the workgroup
    int lda = lda0;
    size_t boff = (size_t)b * bstride;
    if (rag) {   // ragged batch: rows of this matrix end at its own order
        np = min(np, rag[b].live);
        if (c0 + TB + (int)blockIdx.x * TR_ROWS >= np) return;   // uniform
        lda = rag[b].lda;
        boff = rag[b].off;
    }
    __shared__ double lks[TB * TB];
    for (int e = threadIdx.x; e < TB * TB; e += TR_THREADS) lks[e] = lk0[(size_t)b * TB * TB + e];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    constexpr int RB = PT_RB;
    const int r0 = c0 + TB + blockIdx.x * TR_ROWS + 16 * RB * wave;
    if (r0 >= np) return;   // whole waves; after the only barrier
    double *A = A0 + boff;

    // -X_pre^T = -C^T + P_kk P_rows^T
    dbl4 T[4][RB];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const double *p = A + (size_t)(r0 + 16 * rb + li) + (size_t)(c0 + 16 * cb + g) * lda;
            const size_t s4 = (size_t)4 * lda;
            T[cb][rb] = -(dbl4){p[0], p[s4], p[2 * s4], p[3 * s4]};
        }
    if (K > 0) {
        const double *pd = A + (size_t)(c0 + li) + (size_t)(kc0 + g) * lda;
        const double *pr = A + (size_t)(r0 + li) + (size_t)(kc0 + g) * lda;
        const size_t step4 = (size_t)4 * lda;
        // PT_NSETS fragment sets in flight (prefetch distance PT_NSETS
        // k-steps; K is a multiple of 64), each reloaded right after its
        // MFMAs, as in the trailing update; the reloads past the end re-read
        // the set just used (in bounds, unused)
        constexpr int NS = PT_NSETS;
        double fa[NS][4], fb[NS][RB];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
#pragma unroll
            for (int q = 0; q < 4; ++q) fa[st][q] = pd[st * step4 + 16 * q];
#pragma unroll
            for (int q = 0; q < RB; ++q) fb[st][q] = pr[st * step4 + 16 * q];
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int k = 0; k < K; k += 4 * NS) {
#pragma unroll
            for (int st = 0; st < NS; ++st) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        T[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[st][cb], fb[st][rb],
                                                                         T[cb][rb], 0, 0, 0);
                const size_t nx = (k + 4 * (NS + st) < K) ? (size_t)(NS + st) * step4
                                                          : (size_t)st * step4;
#pragma unroll
                for (int q = 0; q < 4; ++q) fa[st][q] = pd[nx + 16 * q];
#pragma unroll
                for (int q = 0; q < RB; ++q) fb[st][q] = pr[nx + 16 * q];
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            }
            pd += NS * step4;
            pr += NS * step4;
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) T[cb][rb] = -T[cb][rb];

#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        // substitution inside column block jb
#pragma unroll
        for (int cp = 0; cp < 16; ++cp) {
            const int e0 = cp >> 2, g0 = cp & 3, c = 16 * jb + cp;
            const double linv = lks[c * TB + c];
            double lm[4];   // L(16 jb + 4 e + g, c) for this lane's elements
#pragma unroll
            for (int e = 0; e < 4; ++e) lm[e] = lks[c * TB + 16 * jb + 4 * e + g];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                double v = T[jb][rb][e0];
                v = (g == g0) ? v * linv : v;
                T[jb][rb][e0] = v;
                const double xc = __shfl(v, li + 16 * g0, 64);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * e + 3 > cp)   // some lane of element e is right of c
                        T[jb][rb][e] = (4 * e + g > cp) ? fma(-xc, lm[e], T[jb][rb][e])
                                                        : T[jb][rb][e];
            }
        }
        // the later column blocks: X^T(cb) -= L(cb, jb) X^T(jb)
#pragma unroll
        for (int cb = jb + 1; cb < 4; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double la = -lks[(16 * jb + 4 * q + g) * TB + 16 * cb + li];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    T[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(la, T[jb][rb][q], T[cb][rb],
                                                                     0, 0, 0);
            }
    }

#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            double *p = A + (size_t)(r0 + 16 * rb + li) + (size_t)(c0 + 16 * cb + g) * lda;
            const size_t s4 = (size_t)4 * lda;
            p[0] = T[cb][rb].x;
            p[s4] = T[cb][rb].y;
            p[2 * s4] = T[cb][rb].z;
            p[3 * s4] = T[cb][rb].w;
        }
}

// ---------------------------------------------------------------------------
// SYRK/GEMM update on FP64 MFMA (v_mfma_f64_16x16x4f64).
// Work item = (matrix, 128 x 128 output tile on or below the diagonal of the
// column range).  Each of the 4 waves owns a 64 x 64 quadrant = 4 x 4 MFMA
// blocks of 16 x 16; quadrants above the diagonal or outside the range idle.
// Operand layout of the 16x16x4 f64 MFMA (wave64, measured on gfx950):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, and D[i][j] in lane
// j + 16 (i % 4), element i / 4.  The A rows are fed permuted,
// MFMA row i <- matrix row 4 (i % 4) + i / 4, so that the four accumulator
// elements of lane l are the four consecutive matrix rows 4 (l / 16) + 0..3
// of column l % 16: C is loaded and stored with 2 x 16-byte accesses per
// lane.  The accumulators start at -C and the chain adds A(r,k) A(c,k), so
// the result C - sum_k A(r,k) A(c,k) is stored with one sign flip.  Two
// fragment sets alternate: each is reloaded for the k-step after next as
// soon as its 16 MFMAs are issued.
// Work items are mapped XCD-major: blocks are dispatched round-robin over the
// 8 XCDs, so block id b runs on XCD b % 8; consecutive work items (same
// matrix) are given to the same XCD and share its L2 for the panel reads.
// Inside a matrix the 128 x 128 tiles go in blocks of SY_SR tile rows x
// SY_SC tile columns (column-major inside a block): the tiles an XCD runs
// at one time (32 CUs x 2 workgroups) then read SY_SR + SY_SC panel blocks
// of 128 rows between them instead of one row block each, so the panel is
// fetched from HBM about (1/SY_SC + 1/SY_SR) times per tile rather than once.

constexpr int SY_THREADS = 256;
constexpr int NXCD = 8;
#ifndef SY_NSETS
#define SY_NSETS 2   // fragment sets in flight (prefetch distance in k-steps of 4)
#endif
#ifndef SY_SR
#define SY_SR 8
#endif
#ifndef SY_SC
#define SY_SC 8
#endif

// Tile t (work order) of the lower 128 x 128 tiles (it >= jt) of NR tile
// rows and NC tile columns, in blocks of SY_SR x SY_SC tiles, column block
// by column block, tiles column-major inside a block.
__device__ __forceinline__ void sy_tile(int t, int NR, int NC, int &it, int &jt)
{
    for (int j0 = 0; j0 < NC; j0 += SY_SC) {
        const int j1 = min(NC, j0 + SY_SC);
        for (int i0 = j0; i0 < NR; i0 += SY_SR) {
            const int i1 = min(NR, i0 + SY_SR);
            int cnt = 0;
            for (int j = j0; j < j1; ++j) cnt += max(0, i1 - max(i0, j));
            if (t < cnt) {
                for (int j = j0; j < j1; ++j) {
                    const int c = max(0, i1 - max(i0, j));
                    if (t < c) {
                        jt = j;
                        it = max(i0, j) + t;
                        return;
                    }
                    t -= c;
                }
            }
            t -= cnt;
        }
    }
    it = jt = NR;   // not reached for t < the tile count (then out of range)
}

// WR x WC waves of 64 x 64: <2,2> = 128 x 128 tiles over a lower-triangular
// column range; <4,1> = 256 x 64 tiles over a single 64-wide column block.
template <int WR, int WC>
__global__ __launch_bounds__(SY_THREADS, 2)
void syrk_update_kernel(double *__restrict__ A0, int lda0, size_t bstride, int np, int cs,
                        int ce, int kc0, int K, int NR, int ntiles, int batch,
                        const uint8_t *__restrict__ mask, const RagMat *__restrict__ rag,
                        int whole)
{
    constexpr int TR = 64 * WR, TC = 64 * WC;
    const int bid = blockIdx.x;
    int b, t, NRb = NR, NCb = WC > 1 ? (ce - cs + TC - 1) / TC : 1;
    int lda = lda0;
    size_t boff;
    if (rag) {
        // ragged batch (matrices in order of decreasing order; the grid has
        // room for the tiles of the largest, ntiles, per matrix):
        // `whole`: matrix b on XCD b % NXCD, whole, so that each XCD's L2
        //   serves one matrix's panel at a time (the host chooses it when
        //   that spreads the tiles evenly over the XCDs);
        // else: matrix b's own tiles cut into NXCD contiguous pieces, piece
        //   x on XCD x, so no XCD idles whatever the sizes.
        const int x = bid % NXCD, local = bid / NXCD;
        int j;
        if (whole) {
            b = x + NXCD * (local / ntiles);
            j = local % ntiles;
        } else {
            const int chunk = (ntiles + NXCD - 1) / NXCD;
            b = local / chunk;
            j = local - b * chunk;
        }
        if (b >= batch) return;
        np = min(np, rag[b].live);
        NRb = (np - cs + TR - 1) / TR;
        if (NRb <= 0) return;
        if (WC > 1) NCb = (min(ce, np) - cs + TC - 1) / TC;
        const int nt = WC > 1 ? NCb * NRb - NCb * (NCb - 1) / 2 : NRb;
        if (whole) {
            t = j;
            if (t >= nt) return;
        } else {
            const int cb = (nt + NXCD - 1) / NXCD;
            t = x * cb + j;
            if (j >= cb || t >= nt) return;
        }
        lda = rag[b].lda;
        boff = rag[b].off;
    } else {
        const int W = ntiles * batch;
        const int per = (W + NXCD - 1) / NXCD;
        const int work = (bid % NXCD) * per + bid / NXCD;
        if (work >= W) return;
        b = work / ntiles;
        if (mask && !mask[b]) return;
        t = work - b * ntiles;
        boff = (size_t)b * bstride;
    }
    int jt = 0, it = t;
    if (WC > 1) {
        if (SY_SC > 0) {
            sy_tile(t, NRb, NCb, it, jt);
        } else {   // column-major over the whole range
            while (t >= NRb - jt) { t -= NRb - jt; ++jt; }
            it = jt + t;
        }
    }

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int r0 = cs + TR * it + 64 * (wave / WC);
    const int c0 = cs + TC * jt + 64 * (wave % WC);
    if (r0 >= np || c0 >= ce || r0 < c0) return;   // no barriers below

    double *A = A0 + boff;
    const int li = lane & 15, lk = lane >> 4;
    const int pli = 4 * (li & 3) + (li >> 2);   // permuted A row of this lane

    // operand pointers; the fragments of the first SY_NSETS k-steps go out first
    const double *pa = A + (size_t)(r0 + pli) + (size_t)(kc0 + lk) * lda;
    const double *pb = A + (size_t)(c0 + li) + (size_t)(kc0 + lk) * lda;
    const size_t step4 = (size_t)4 * lda;
    // (in set order, before the loads of C: the loop then finds set 0's
    // fragments the oldest loads in flight on entry as on every later trip)
    double fa[SY_NSETS][4], fb[SY_NSETS][4];
#pragma unroll
    for (int st = 0; st < SY_NSETS; ++st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            fa[st][q] = pa[st * step4 + 16 * q];
            fb[st][q] = pb[st * step4 + 16 * q];
        }
        __builtin_amdgcn_sched_barrier(0);
    }

    // accumulators start at -C and gather +A(r,k) A(c,k): no per-step negation
    dbl4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double *p = A + (size_t)(r0 + 16 * rb + 4 * lk) + (size_t)(c0 + 16 * cb + li) * lda;
            dbl2 lo = *(const dbl2 *)p;
            dbl2 hi = *(const dbl2 *)(p + 2);
            acc[rb][cb] = -(dbl4){lo.x, lo.y, hi.x, hi.y};
        }

    // K is a multiple of 4 SY_NSETS: SY_NSETS k-steps per trip, each
    // fragment set reloaded for the trip after this one right after its
    // MFMAs were issued (prefetch distance SY_NSETS k-steps).  The reloads
    // are unconditional (in the last trip they re-read the set just used, in
    // bounds and unused), so every trip issues the same loads and each set
    // waits only for its own fragments, not for the whole prefetch queue.
    for (int kk = 0; kk < K; kk += 4 * SY_NSETS) {
#pragma unroll
        for (int st = 0; st < SY_NSETS; ++st) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[st][rb], fb[st][cb],
                                                                       acc[rb][cb], 0, 0, 0);
            const size_t nx = (kk + 4 * (SY_NSETS + st) < K) ? (size_t)(SY_NSETS + st) * step4
                                                              : (size_t)st * step4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fa[st][q] = pa[nx + 16 * q];
                fb[st][q] = pb[nx + 16 * q];
            }
            // keeps these loads here: without the memory barrier the compiler
            // merges them with the prologue loads into one load at the top of
            // the loop, right before the first use; without the scheduling
            // barrier it moves them below the later sets' MFMAs
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
        pa += SY_NSETS * step4;
        pb += SY_NSETS * step4;
    }

#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            double *p = A + (size_t)(r0 + 16 * rb + 4 * lk) + (size_t)(c0 + 16 * cb + li) * lda;
            dbl4 v = -acc[rb][cb];
            *(dbl2 *)p = (dbl2){v.x, v.y};
            *(dbl2 *)(p + 2) = (dbl2){v.z, v.w};
        }
}

// Trailing update with FP32 MFMA (v_mfma_f32_16x16x4f32) and FP32
// accumulation, for the mixed-precision mode: the FP64 panel fragments are
// rounded to FP32, the product sum over K is accumulated in FP32, and the
// result is subtracted from the FP64 matrix in FP64.  Layout of the f32
// MFMA (measured on gfx950): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in lane j + 16 (i / 4), element i % 4, so each lane's four
// accumulator elements are four consecutive rows without permutation.
typedef float flt4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(SY_THREADS, 2)
void syrk_update_f32_kernel(double *__restrict__ A0, int lda, size_t bstride, int np, int cs,
                            int ce, int kc0, int K, int NR, int ntiles, int batch,
                            const uint8_t *__restrict__ mask)
{
    const int W = ntiles * batch;
    const int per = (W + NXCD - 1) / NXCD;
    const int bid = blockIdx.x;
    const int work = (bid % NXCD) * per + bid / NXCD;
    if (work >= W) return;
    const int b = work / ntiles;
    if (mask && !mask[b]) return;
    int t = work - b * ntiles;
    int jt = 0;
    while (t >= NR - jt) { t -= NR - jt; ++jt; }
    const int it = jt + t;

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int r0 = cs + 128 * it + 64 * (wave >> 1);
    const int c0 = cs + 128 * jt + 64 * (wave & 1);
    if (r0 >= np || c0 >= ce || r0 < c0) return;   // no barriers below

    double *A = A0 + (size_t)b * bstride;
    const int li = lane & 15, lk = lane >> 4;
    const double *pa = A + (size_t)(r0 + li) + (size_t)(kc0 + lk) * lda;
    const double *pb = A + (size_t)(c0 + li) + (size_t)(kc0 + lk) * lda;
    const size_t step4 = (size_t)4 * lda;
    double a0[4], b0[4], a1[4], b1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { a0[q] = pa[16 * q]; b0[q] = pb[16 * q]; }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) { a1[q] = pa[step4 + 16 * q]; b1[q] = pb[step4 + 16 * q]; }
    __builtin_amdgcn_sched_barrier(0);

    flt4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = (flt4){0.f, 0.f, 0.f, 0.f};

    for (int kk = 0; kk < K; kk += 8) {
        float fa[4], fb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) { fa[q] = (float)a0[q]; fb[q] = (float)b0[q]; }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[rb], fb[cb], acc[rb][cb], 0, 0, 0);
        // the reloads are unconditional (in the last trip they re-read the
        // fragments just used, in bounds and unused) and pinned in place, so
        // each half-trip waits for its own loads only (as in the FP64 kernel)
        const size_t n0 = (kk + 8 < K) ? 2 * step4 : 0, n1 = (kk + 12 < K) ? 2 * step4 : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) { a0[q] = pa[n0 + 16 * q]; b0[q] = pb[n0 + 16 * q]; }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) { fa[q] = (float)a1[q]; fb[q] = (float)b1[q]; }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[rb], fb[cb], acc[rb][cb], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) { a1[q] = pa[n1 + step4 + 16 * q]; b1[q] = pb[n1 + step4 + 16 * q]; }
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        pa += 2 * step4;
        pb += 2 * step4;
    }

    // C is read whole before the first store (the stores might alias later
    // loads as far as the compiler knows, which would serialise them)
    dbl2 cv[4][4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double *p = A + (size_t)(r0 + 16 * rb + 4 * lk) + (size_t)(c0 + 16 * cb + li) * lda;
            cv[rb][cb][0] = *(const dbl2 *)p;
            cv[rb][cb][1] = *(const dbl2 *)(p + 2);
        }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            double *p = A + (size_t)(r0 + 16 * rb + 4 * lk) + (size_t)(c0 + 16 * cb + li) * lda;
            const dbl2 lo = cv[rb][cb][0], hi = cv[rb][cb][1];
            const flt4 v = acc[rb][cb];
            *(dbl2 *)p = (dbl2){lo.x - (double)v.x, lo.y - (double)v.y};
            *(dbl2 *)(p + 2) = (dbl2){hi.x - (double)v.z, hi.y - (double)v.w};
        }
}

__global__ void logdet_sum_kernel(const double *__restrict__ lpart, int nparts, int batch,
                                  double *__restrict__ logdet)
{
    const int b = blockIdx.x;
    double v = 0.0;
    for (int q = threadIdx.x; q < nparts; q += 64) v += lpart[(size_t)b * nparts + q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) logdet[b] = v;
}

}  // namespace

// (ragged launches report the figures of the largest matrix for every one)
void launch_potrf_diag(double *A, int lda, size_t bstride, int c0, int kc0, int K, int batch,
                       int32_t *info, double *lpart, int nparts, double *lk, hipStream_t s,
                       const uint8_t *mask, const RagMat *rag)
{
    ProfScope ps(K_POTRF_DIAG, (TB * TB * TB / 3.0 + 2.0 * TB * TB * K) * batch,
                 (16.0 * TB * TB + 8.0 * TB * K) * batch, s);
    potrf_diag_kernel<<<batch, PO_THREADS, 0, s>>>(A, lda, bstride, c0, kc0, K, info, lpart,
                                                   nparts, lk, mask, rag);
}

void launch_panel_trsm(double *A, int lda, size_t bstride, int np, int c0, int kc0, int K,
                       int batch, const double *lk, hipStream_t s, const uint8_t *mask,
                       const RagMat *rag)
{
    int rows = np - (c0 + TB);
    if (rows <= 0) return;
    // update 2 rows 64 K, substitution rows 64^2; bytes: the block in and
    // out, the panel rows and L_kk
    ProfScope ps(K_TRSM_PANEL, ((double)rows * TB * TB + 2.0 * rows * TB * K) * batch,
                 (16.0 * rows * TB + 8.0 * rows * K + 8.0 * TB * TB) * batch, s);
    dim3 grid((rows + TR_ROWS - 1) / TR_ROWS, batch);
    panel_trsm_kernel<<<grid, TR_THREADS, 0, s>>>(A, lda, bstride, np, c0, kc0, K, lk, mask, rag);
}

void launch_syrk_update(double *A, int lda, size_t bstride, int np, int cs, int ce, int kc0,
                        int K, int batch, hipStream_t s, int prec, const uint8_t *mask,
                        const RagMat *rag, const int32_t *hlive)
{
    if (ce <= cs || K <= 0) return;
    const double entries = (double)(ce - cs) * np - 0.5 * (double)(cs + ce - 1) * (ce - cs);
    // left-looking updates of one 64-column block inside an outer panel are
    // reported apart from the rank-OUTER_NB trailing updates
    const bool block64 = (ce - cs) == TB;
    const bool f32 = !block64 && prec == GP_MIXED_FAST;
    ProfScope ps(block64 ? K_SYRK_PANEL : (f32 ? K_SYRK_UPDATE_F32 : K_SYRK_UPDATE),
                 2.0 * K * entries * batch,
                 (16.0 * entries + 8.0 * (double)(np - cs) * K) * batch, s);
    int NR, ntiles;
    if (block64) {
        NR = (np - cs + 255) / 256;
        ntiles = NR;
    } else {
        NR = (np - cs + 127) / 128;
        const int NC = (ce - cs + 127) / 128;
        ntiles = 0;
        for (int jt = 0; jt < NC; ++jt) ntiles += NR - jt;
    }
    const long W = (long)ntiles * batch;
    // ragged: whole matrices round-robin over the XCDs when that loads every
    // XCD within 10% of the mean (from the host copy of the orders), else
    // NXCD pieces of the largest matrix's tile count per matrix
    long per = (W + NXCD - 1) / NXCD;
    int whole = 0;
    if (rag) {
        if (hlive && batch >= NXCD) {
            const int TR = block64 ? 256 : 128, TC = block64 ? 64 : 128;
            long load[NXCD] = {}, tot = 0;
            for (int b = 0; b < batch; ++b) {
                const int nb_ = min(np, (int)hlive[b]);
                const int nr = (nb_ - cs + TR - 1) / TR;
                if (nr <= 0) continue;
                const int nc = block64 ? 1 : (min(ce, nb_) - cs + TC - 1) / TC;
                const long nt = block64 ? nr : (long)nc * nr - (long)nc * (nc - 1) / 2;
                load[b % NXCD] += nt;
                tot += nt;
            }
            long mx = 0;
            for (int x = 0; x < NXCD; ++x) mx = max(mx, load[x]);
            whole = mx * NXCD <= tot + tot / 10;
        }
        per = whole ? (long)ntiles * ((batch + NXCD - 1) / NXCD)
                    : (long)((ntiles + NXCD - 1) / NXCD) * batch;
    }
    if (block64)
        syrk_update_kernel<4, 1><<<(unsigned)(per * NXCD), SY_THREADS, 0, s>>>(
            A, lda, bstride, np, cs, ce, kc0, K, NR, ntiles, batch, mask, rag, whole);
    else if (f32)
        syrk_update_f32_kernel<<<(unsigned)(per * NXCD), SY_THREADS, 0, s>>>(
            A, lda, bstride, np, cs, ce, kc0, K, NR, ntiles, batch, mask);
    else
        syrk_update_kernel<2, 2><<<(unsigned)(per * NXCD), SY_THREADS, 0, s>>>(
            A, lda, bstride, np, cs, ce, kc0, K, NR, ntiles, batch, mask, rag, whole);
}

namespace {

// Side streams (and their events) of one caller stream, created on first use
// per (device, caller stream) and kept until release_side_streams(caller)
// (the request server calls it for each of its streams before destroying
// them) or the end of the process: `s` for the lookahead trailing updates,
// `solve` for the solve segments.  Default
// priority, non-blocking.  At most SIDE_CALLERS caller streams get them;
// calls on further streams factor without the lookahead (same results), so a
// caller that cycles through new streams does not make the library create
// streams without bound.
constexpr size_t SIDE_CALLERS = 64;
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipStream_t solve = nullptr;
    hipEvent_t panel = nullptr, solved = nullptr;
};

std::mutex side_mu;
std::map<std::pair<int, hipStream_t>, SideStream> side_table;

SideStream *side_for(hipStream_t caller)
{
    std::mutex &mu = side_mu;
    auto &table = side_table;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, caller);
    auto it = table.find(key);
    if (it != table.end()) return it->second.s ? &it->second : nullptr;
    if (table.size() >= SIDE_CALLERS) return nullptr;
    SideStream sd;
    if (hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&sd.solve, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sd.panel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sd.solved, hipEventDisableTiming) != hipSuccess) {
        // no lookahead for this stream; free what was made, remember the failure
        for (hipEvent_t e : {sd.fork, sd.join, sd.panel, sd.solved})
            if (e) (void)hipEventDestroy(e);
        for (hipStream_t st : {sd.s, sd.solve})
            if (st) (void)hipStreamDestroy(st);
        (void)hipGetLastError();
        table[key] = SideStream{};
        return nullptr;
    }
    table[key] = sd;
    return &table[key];
}

}  // namespace

void release_side_streams(hipStream_t caller)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(side_mu);
    auto it = side_table.find(std::make_pair(dev, caller));
    if (it == side_table.end()) return;
    SideStream &sd = it->second;
    if (sd.s) {
        (void)hipStreamSynchronize(sd.s);
        (void)hipStreamSynchronize(sd.solve);
        (void)hipEventDestroy(sd.fork);
        (void)hipEventDestroy(sd.join);
        (void)hipEventDestroy(sd.panel);
        (void)hipEventDestroy(sd.solved);
        (void)hipStreamDestroy(sd.s);
        (void)hipStreamDestroy(sd.solve);
    }
    side_table.erase(it);
}

// Blocked right-looking Cholesky with a one-panel lookahead: after outer
// panel [c, pe) is factored, the trailing update is split at the end of the
// next panel.  The next panel's columns are updated on the caller's stream
// and factored there while the rest of the trailing matrix is updated on a
// side stream; the caller's stream waits for that update before it touches
// the same columns (the next trailing update).  The two streams write
// disjoint column ranges and read only finished panels, so the result is the
// same operations in the same order per entry as without the lookahead.
// With a solve plan, each finished panel's columns of the forward solve run on
// a third stream (after an event on the caller's stream marks the panel
// done) while the next panels are factored; the caller's stream waits for
// the last segment.  Without side streams the whole solve follows the
// factorisation on the caller's stream.  The segments are the same
// operations in the same order as one whole solve.
void factor_batch(double *A, int lda, size_t bstride, int np, int batch, int32_t *info,
                  double *lpart, double *lk, hipStream_t s, int prec, bool bordered,
                  const uint8_t *mask, int8_t *crt_res, int32_t *crt_ex, bool lookahead,
                  int extra, const SolvePlan *plan, const RagMat *rag, const int32_t *hlive)
{
    const int nparts = np / TB;
    // ragged batch: the matrices come in order of decreasing order (hlive:
    // host copy of their `live`), so those a launch at column x still has to
    // touch (live > x) are the first act(x); the launch covers only them
    auto act = [&](int x) {
        if (!hlive) return batch;
        int lo = 0, hi = batch;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (hlive[mid] > x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    // GP_MIXED: wider panels, the rank of its INT8 trailing updates
    const int nb = prec == GP_MIXED ? GP_MIXED_RANK : OUTER_NB;
    SideStream *sd = lookahead && (bordered || np > 2 * nb) ? side_for(s) : nullptr;
    bool pending = false;   // the side stream holds an update not yet joined
    for (int c = 0; c < np; c += nb) {
        const int pe = min(c + nb, np);
        for (int c0 = c; c0 < pe; c0 += TB) {
            // rows that can be nonzero in column block c0: with a border, row
            // np + i is zero left of column i, so rows up to np + c0 + 63
            const int rmax = bordered ? np + c0 + TB : np + extra;
            // left-looking inside the outer panel: bring block c0 up to date
            // with the blocks [c, c0) of the same panel, then factor it
            // left-looking inside the outer panel: block c0 is brought up to
            // date with the blocks [c, c0) of the same panel by the two
            // kernels that factor it (diagonal tile, then the rows below)
            const int bc = act(c0), bt = act(c0 + TB);
            if (bc == 0) break;
            launch_potrf_diag(A, lda, bstride, c0, c, c0 - c, bc, info, lpart, nparts, lk, s, mask,
                              rag);
            if (bt > 0)
                launch_panel_trsm(A, lda, bstride, rmax, c0, c, c0 - c, bt, lk, s, mask, rag);
        }
        if (plan && sd) {
            // columns [c, pe) of L are final: their part of the forward solve
            (void)hipEventRecord(sd->panel, s);
            (void)hipStreamWaitEvent(sd->solve, sd->panel, 0);
            launch_solve_segment(A, lda, bstride, np, plan->n, plan->y, lpart, nparts, info, act(c),
                                 plan->out, plan->z, c / TB, pe / TB, sd->solve, plan->rag);
        }
        // right-looking rank-(pe - c) update of the trailing matrix: rows up
        // to rlim, columns [pe, cend); with a border it also covers the
        // border columns np .. np + pe - 1
        const int rlim = bordered ? np + pe : np + extra;
        const int cend = bordered ? np + pe : np;
        const int bu = act(pe);
        if (cend <= pe || bu == 0) continue;
        if (pending) {
            (void)hipStreamWaitEvent(s, sd->join, 0);
            pending = false;
        }
        const int K = pe - c;
        const bool mixed = prec == GP_MIXED && !bordered && extra == 0 && crt_res && crt_ex;
        const CrtConst *cc = mixed ? crt_constants(K) : nullptr;
        if (cc) launch_crt_split(A, lda, bstride, np, pe, c, K, bu, *cc, crt_res, crt_ex, s, mask);
        const int upd_prec = prec == GP_MIXED ? GP_FP64 : prec;
        auto update = [&](int cs, int ce, hipStream_t st) {
            if (ce <= cs) return;
            if (cc)
                launch_syrk_update_crt(A, lda, bstride, np, pe, cs, ce, K, bu, *cc, crt_res,
                                       crt_ex, st, mask);
            else
                launch_syrk_update(A, lda, bstride, rlim, cs, ce, c, K, bu, st, upd_prec, mask,
                                   rag, hlive);
        };
        const int sp = min(pe + nb, np);   // end of the next panel
        if (sd && cend > sp && sp > pe) {
            update(pe, sp, s);
            (void)hipEventRecord(sd->fork, s);
            (void)hipStreamWaitEvent(sd->s, sd->fork, 0);
            update(sp, cend, sd->s);
            (void)hipEventRecord(sd->join, sd->s);
            pending = true;
        } else
            update(pe, cend, s);
    }
    if (pending) (void)hipStreamWaitEvent(s, sd->join, 0);
    if (plan && sd) {
        (void)hipEventRecord(sd->solved, sd->solve);
        (void)hipStreamWaitEvent(s, sd->solved, 0);
    } else if (plan) {
        launch_solve_segment(A, lda, bstride, np, plan->n, plan->y, lpart, nparts, info, batch,
                             plan->out, plan->z, 0, np / TB, s, plan->rag);
    }
}

void launch_logdet_sum(const double *lpart, int nparts, int batch, double *logdet, hipStream_t s)
{
    ProfScope ps(K_LOGDET_SUM, (double)nparts * batch, 8.0 * (nparts + 1) * batch, s);
    logdet_sum_kernel<<<batch, 64, 0, s>>>(lpart, nparts, batch, logdet);
}

}  // namespace gpk
