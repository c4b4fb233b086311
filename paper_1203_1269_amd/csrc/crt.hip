// Matched-accuracy trailing update on INT8 MFMA by modular arithmetic
// (GP_MIXED).
//
// The rank-K update C -= P P^T of the blocked Cholesky (P: the m x K block of
// the factor below a finished outer panel) is formed exactly in integers and
// rounded once, by the Chinese remainder theorem (the modular variant of the
// Ozaki scheme; Ozaki, Uchino & Imamura, "Ozaki Scheme II: a GEMM-oriented
// emulation of floating-point matrix multiplication using an integer modular
// technique", 2025), written here from that description:
//   * every row i of P gets a power-of-two scale 2^e_i > max_k |P_ik| and is
//     rounded to the integers a_ik = rint(P_ik 2^(b - e_i)), |a_ik| <= 2^b;
//     b is chosen so that K 2^(2b) <= M / 4, M = m_1 ... m_N;
//   * S = a a^T is an integer matrix with |S_ij| <= K 2^(2b) <= M/4; for each
//     modulus m_l the residue matrix A_l = a mod m_l (symmetric range, INT8)
//     gives A_l A_l^T, exact in INT32 on v_mfma_i32_16x16x64_i8, whose
//     residue c_l = (A_l A_l^T) mod m_l equals S mod m_l;
//   * S / M = sum_l c_l y_l / m_l (mod 1), y_l = (M / m_l)^-1 mod m_l.  Each
//     fraction y_l / m_l is split as f1_l + f2_l with f1_l a multiple of
//     2^-40: the sum of c_l f1_l is exact in FP64 (|c_l| < 2^8, 16 terms)
//     and is reduced mod 1 exactly; the sum of c_l f2_l (below 2^-28) is
//     rounded at 2^-80; the centred fraction times M 2^(-2b) 2^(e_i + e_j) is
//     the update entry, subtracted from C in FP64.
// The only approximation is the rounding of P to b fraction bits per row
// (b = 56 at K = 768 with the sixteen moduli below): an entry's error is at
// most 2^(e_i + e_j - b) K, against the K u 2^(e_i + e_j) bound of an FP64
// product (u = 2^-53), so the update is as accurate as the FP64 one.
//
// Sixteen INT8 products per FP64 product (against 64 FP64 MFMA cycles per
// 16x16x4 block, one 16x16x64 INT8 MFMA takes 16): a 2.2x MFMA-cycle
// advantage over FP64 before the reduction work.
#include <math.h>

#include <mutex>

#include "kernels.hpp"

namespace gpk {

namespace {

// Pairwise coprime moduli, largest first: 2^8 and odd numbers <= 255, so a
// symmetric residue fits INT8 and |residue|^2 K <= 2^24 for K <= 1024.
constexpr int CRT_MODULI[CRT_NMOD] = {256, 255, 253, 251, 247, 241, 239, 233,
                                      229, 227, 223, 217, 211, 199, 197, 193};

typedef int int4v __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// Byte offset of the 1 KiB fragment (modulus l, 64-deep k chunk kc, 16-row
// block rb) in one theta's residues: modulus-major, then chunk, then row
// block, so the row blocks of one (l, kc) are one contiguous run.  Within a
// fragment lane L holds row L % 16 and k bytes 16 (L / 16) .. + 15 (the
// operand layout of v_mfma_i32_16x16x64_i8).
__host__ __device__ inline size_t crt_frag_off(int l, int kc, int rb, int KC, int nrb)
{
    return (((size_t)l * KC + kc) * nrb + rb) * 1024;
}

// ---------------------------------------------------------------------------
// Split: per row the exponent e_i and, for each modulus, the residues of
// a_ik = rint(P_ik 2^(b - e_i)).  One workgroup per 16 rows of P; wave w
// covers k chunks w, w + 4, ...; lane L row L % 16 and k bytes 16 (L / 16)
// .. + 15 of each chunk.  a is split exactly as a_hi 2^29 + a_lo (|a_hi|,
// |a_lo| <= 2^28), so a mod m = (a_hi (2^29 mod m) + a_lo) mod m is formed on
// integers below 2^37 in FP64 and reduced by one rounded division (exact
// nearest integer: the quotient estimate is within 2^-20 and m has no
// half-integer quotients except m = 256, where the +-128 tie wraps to the
// same INT8 byte).
template <int CPW>
__global__ __launch_bounds__(256)
void crt_split_kernel(const double *__restrict__ A0, int lda, size_t bstride, int pe, int kc0,
                      int nrb, CrtConst cc, int8_t *__restrict__ sl0, size_t sl_stride,
                      int32_t *__restrict__ ex0, int ex_stride, const uint8_t *__restrict__ mask)
{
    const int b = blockIdx.y;
    if (mask && !mask[b]) return;   // uniform over the workgroup
    __shared__ double wmax[4][16];
    const int rb = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = 16 * rb + (lane & 15);           // row of P (0 .. m-1)
    const double *A = A0 + (size_t)b * bstride + (size_t)(pe + row) +
                      (size_t)(kc0 + 64 * wave + 16 * (lane >> 4)) * lda;
    double v[CPW][16];
    double mx = 0.0;
#pragma unroll
    for (int h = 0; h < CPW; ++h)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            v[h][q] = A[(size_t)(256 * h + q) * lda];   // chunk wave + 4 h
            mx = fmax(mx, fabs(v[h][q]));
        }
    mx = fmax(mx, __shfl_xor(mx, 16, 64));
    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    if (lane < 16) wmax[wave][lane] = mx;
    __syncthreads();
    mx = fmax(fmax(wmax[0][lane & 15], wmax[1][lane & 15]),
              fmax(wmax[2][lane & 15], wmax[3][lane & 15]));
    int e;
    (void)frexp(mx, &e);   // mx < 2^e (e = 0 for an all-zero row)
    if (wave == 0 && lane < 16) ex0[(size_t)b * ex_stride + row] = e;

    const int KC = CPW * 4;
    int8_t *sl = sl0 + (size_t)b * sl_stride + (size_t)lane * 16;
#pragma unroll
    for (int h = 0; h < CPW; ++h) {
        double ahi[16], alo[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const double a = rint(ldexp(v[h][q], cc.b - e));   // |a| <= 2^b, exact
            ahi[q] = rint(a * 0x1p-29);
            alo[q] = fma(-ahi[q], 0x1p29, a);                   // exact, |alo| <= 2^28
        }
        const int kc = wave + 4 * h;
        for (int l = 0; l < CRT_NMOD; ++l) {
            const double m = cc.md[l], inv = cc.invd[l], t = cc.t29[l];
            int4v w;
#pragma unroll
            for (int word = 0; word < 4; ++word) {
                uint32_t packed = 0;
#pragma unroll
                for (int byte = 0; byte < 4; ++byte) {
                    const int q = 4 * word + byte;
                    const double s = fma(ahi[q], t, alo[q]);   // exact, |s| < 2^37
                    const double r = fma(-rint(s * inv), m, s);  // s mod m, symmetric
                    packed |= ((uint32_t)(int)r & 0xffu) << (8 * byte);
                }
                w[word] = (int)packed;
            }
            *(int4v *)(sl + crt_frag_off(l, kc, rb, KC, nrb)) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// Update: C -= P P^T over 128 x 128 tiles of the trailing matrix (rows and
// columns local to pe), column range [cs, ce) (local), lower tiles only.
// Eight waves (two per SIMD): wave w owns rows 64 (w / 4) .. + 63 and columns
// 32 (w % 4) .. + 31 of the tile, a 4 x 2 grid of 16 x 16 MFMA blocks.  The
// residues of the tile's 128 rows and 128 columns for CRT_CPB consecutive
// (modulus, 64-deep k chunk) pairs form one LDS stage (16 fragments of 1 KiB
// per chunk), copied by global_load_lds_dwordx4 (two fragments per wave and
// chunk) CRT_NST - 1 stages ahead; a stage is overwritten only after the
// barrier that follows its last use, and all fragment reads of a chunk are
// issued before the MFMAs of the chunk before it.  After the K / 64 chunks of
// one modulus the INT32 accumulators are reduced mod m_l (FP64, exact) and
// folded into the per-entry fractions hi (exact, multiples of 2^-40) and lo;
// after the last modulus each entry is centred, scaled by
// M 2^(e_i + e_j - 2b) and subtracted from C.  Waves of the tile above the
// diagonal (64-row blocks) or outside the matrix skip the MFMAs and the store
// but take part in the copies and barriers.
//
// Work order: the operands are 16 bytes per entry of P (twice the FP64
// panel), so reuse in the 4 MB L2 of an XCD decides the speed.  Work items
// go to the XCDs in contiguous ranges (block b runs on XCD b % 8), and within
// one matrix the tiles are taken in blocks of CRT_SR tile rows x CRT_SC tile
// columns: the 32 workgroups that run at once on an XCD then share CRT_SR row
// slabs and CRT_SC column slabs of residues instead of streaming one row slab
// each.
constexpr int CRT_THREADS = 512;
#ifndef CRT_NST
#define CRT_NST 4
#endif
#ifndef CRT_CPB
#define CRT_CPB 2
#endif
#ifndef CRT_SR
#define CRT_SR 8
#endif
#ifndef CRT_SC
#define CRT_SC 4
#endif
constexpr int NXCD_CRT = 8;

template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    // s_waitcnt with vmcnt = N (bits 3:0 and 15:14), expcnt and lgkmcnt not waited for
    __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

#define LDS_AS __attribute__((address_space(3)))

// Tile t (0-based, in work order) of the lower tiles of tile columns
// [jt0, jt1) and tile rows [jt, NT): blocks of SR tile rows x SC tile
// columns, column block by column block, tiles column-major inside a block.
__device__ __forceinline__ void crt_tile(int t, int NT, int jt0, int jt1, int &it, int &jt)
{
    for (int j0 = jt0; j0 < jt1; j0 += CRT_SC) {
        const int j1 = min(jt1, j0 + CRT_SC);
        for (int i0 = j0 - (j0 - jt0) % CRT_SR; i0 < NT; i0 += CRT_SR) {
            const int i1 = min(NT, i0 + CRT_SR);
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
    it = jt = -1;   // not reached for t < the tile count
}

template <int NST, int CPB>
__global__ __launch_bounds__(CRT_THREADS, 1)
void syrk_update_crt_kernel(double *__restrict__ A0, int lda, size_t bstride, int pe, int m,
                            int ce_loc, int jt0, int jt1, int NT, int ntiles, int batch, int KC,
                            int nrb, CrtConst cc, const int8_t *__restrict__ sl0,
                            size_t sl_stride, const int32_t *__restrict__ ex0, int ex_stride,
                            const uint8_t *__restrict__ mask)
{
    __shared__ __attribute__((aligned(1024))) int8_t stage[NST][CPB * 16384];
    const int W = ntiles * batch;
    const int per = (W + NXCD_CRT - 1) / NXCD_CRT;
    const int bid = blockIdx.x;
    const int work = (bid % NXCD_CRT) * per + bid / NXCD_CRT;
    if (work >= W) return;   // uniform over the workgroup, before any copy
    const int b = work / ntiles;
    if (mask && !mask[b]) return;
    int it, jt;
    crt_tile(work - b * ntiles, NT, jt0, jt1, it, jt);
    if (it < 0) return;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = 128 * it + 64 * (wave >> 2);
    const int c0 = 128 * jt + 32 * (wave & 3);
    const bool active = r0 < m && c0 < ce_loc && (r0 >> 6) >= (c0 >> 6);

    // this wave's two fragments of every chunk: tile fragments 2w, 2w + 1
    // (0..7: row blocks 8 it .. 8 it + 7, 8..15: column blocks 8 jt ..)
    const int f0 = 2 * wave;
    const int8_t *src = sl0 + (size_t)b * sl_stride + (size_t)lane * 16 +
                        (size_t)(f0 < 8 ? 8 * it + f0 : 8 * jt + f0 - 8) * 1024;
    const size_t cstep = (size_t)nrb * 1024;   // next chunk (and next modulus) in the layout
    const int nsteps = CRT_NMOD * KC / CPB;
    auto issue = [&](int s) {
        const int ss = min(s, nsteps - 1);   // past the end: a harmless re-read
#pragma unroll
        for (int c = 0; c < CPB; ++c) {
            const int8_t *sp = src + (size_t)(ss * CPB + c) * cstep;
            LDS_AS int8_t *dp = (LDS_AS int8_t *)&stage[s % NST][c * 16384 + wave * 2048];
            __builtin_amdgcn_global_load_lds((const void *)sp, (LDS_AS void *)dp, 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(sp + 1024), (LDS_AS void *)(dp + 1024),
                                             16, 0, 0);
        }
    };
#pragma unroll
    for (int s = 0; s < NST - 1; ++s) issue(s);

    double hi[4][2][4], lo[4][2][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) { hi[p][q][e] = 0.0; lo[p][q][e] = 0.0; }
    const int aoff = (wave >> 2) * 4096 + lane * 16;         // my 64 rows: 4 fragments
    const int boff = 8192 + (wave & 3) * 2048 + lane * 16;   // my 32 columns: 2 fragments
    int4v acc[4][2];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = (int4v){0, 0, 0, 0};
    int kc = 0, l = 0;
    for (int s = 0; s < nsteps; ++s) {
        wait_vmcnt<2 * CPB * (NST - 2)>();   // this wave's copies of stage s have landed
        __builtin_amdgcn_s_barrier();        // ... and every other wave's
        issue(s + NST - 1);                  // into the stage read at s - 1
        const int8_t *sb = stage[s % NST];
        int4v fa[2][4], fb[2][2];
#pragma unroll
        for (int p = 0; p < 4; ++p) fa[0][p] = *(const int4v *)(sb + aoff + p * 1024);
#pragma unroll
        for (int q = 0; q < 2; ++q) fb[0][q] = *(const int4v *)(sb + boff + q * 1024);
#pragma unroll
        for (int c = 0; c < CPB; ++c) {
            const int cur = c & 1;
            if (c + 1 < CPB) {   // the next chunk's fragments go out before these MFMAs
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    fa[cur ^ 1][p] = *(const int4v *)(sb + (c + 1) * 16384 + aoff + p * 1024);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    fb[cur ^ 1][q] = *(const int4v *)(sb + (c + 1) * 16384 + boff + q * 1024);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (active) {
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[cur][p], fb[cur][q],
                                                                          acc[p][q], 0, 0, 0);
            }
            if (++kc == KC) {   // modulus l done: fold its residues into the fractions
                kc = 0;
                if (active) {
                    const double md = cc.md[l], inv = cc.invd[l], f1 = cc.f1[l], f2 = cc.f2[l];
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int q = 0; q < 2; ++q)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const double x = (double)acc[p][q][e];        // |x| <= 2^24
                                const double r = fma(-rint(x * inv), md, x);  // x mod m_l, |r| <= 128
                                hi[p][q][e] = fma(r, f1, hi[p][q][e]);        // exact
                                lo[p][q][e] = fma(r, f2, lo[p][q][e]);
                            }
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 2; ++q) acc[p][q] = (int4v){0, 0, 0, 0};
                ++l;
            }
        }
    }
    wait_vmcnt<0>();   // no copy into this workgroup's LDS may outlive it
    if (!active) return;

    // D[i][j] of block (p, q): lane j + 16 (i / 4), element i % 4, i.e. row
    // r0 + 16 p + 4 (lane / 16) + e, column c0 + 16 q + lane % 16
    const int32_t *ex = ex0 + (size_t)b * ex_stride;
    double *A = A0 + (size_t)b * bstride + (size_t)pe + (size_t)pe * lda;
    int eJ[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) eJ[q] = ex[c0 + 16 * q + (lane & 15)];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int row = r0 + 16 * p + 4 * (lane >> 4);
        const int4v eI = *(const int4v *)(ex + row);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            double *pc = A + (size_t)row + (size_t)(c0 + 16 * q + (lane & 15)) * lda;
            const dbl2 v0 = *(const dbl2 *)pc, v1 = *(const dbl2 *)(pc + 2);
            double out[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double h = hi[p][q][e] - rint(hi[p][q][e]);   // exact, in [-1/2, 1/2]
                double x = h + lo[p][q][e];
                x -= rint(x);                                        // S / M, centred
                out[e] -= ldexp(cc.Mscaled * x, eI[e] + eJ[q]);
            }
            *(dbl2 *)pc = (dbl2){out[0], out[1]};
            *(dbl2 *)(pc + 2) = (dbl2){out[2], out[3]};
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host constants of the modular reconstruction for rank K.

bool crt_setup(int K, CrtConst &c)
{
    if (K < 64 || K > 1024 || K % 256 != 0) return false;
    typedef unsigned __int128 u128;
    u128 M = 1;
    for (int l = 0; l < CRT_NMOD; ++l) M *= (u128)CRT_MODULI[l];
    // largest b with K 2^(2b) <= M / 4
    int b = 0;
    while (b < 62 && ((u128)K << (2 * (b + 1))) <= M / 4) ++b;
    c.b = b;
    c.Mscaled = ldexp((double)M, -2 * b);
    for (int l = 0; l < CRT_NMOD; ++l) {
        const int m = CRT_MODULI[l];
        const int Ml = (int)((M / (u128)m) % (u128)m);
        int y = 0;
        for (int t = 1; t < m; ++t)
            if ((Ml * t) % m == 1) { y = t; break; }
        // f_l = y / m = f1 + f2, f1 = N1 2^-40 with N1 = round(y 2^40 / m)
        const long long num = (long long)y << 40;
        const long long N1 = (num + m / 2) / m;
        c.f1[l] = ldexp((double)N1, -40);
        c.f2[l] = (double)(num - N1 * m) / ((double)m * 0x1p40);
        c.mf[l] = (float)m;
        c.inv[l] = 1.0f / (float)m;
        c.md[l] = (double)m;
        c.invd[l] = 1.0 / (double)m;
        c.t29[l] = (double)((1LL << 29) % m);
    }
    return true;
}

// Residues of one theta: CRT_NMOD x K/64 chunks x nrb 16-row fragments with
// the rows of the trailing matrix padded to a multiple of 128 (the update
// reads whole 128-row slabs; rows past the matrix are read, never used).
static inline int crt_nrb(int m) { return 8 * ((m + 127) / 128); }
static inline size_t crt_theta_bytes(int np, int K) { return (size_t)CRT_NMOD * K * 16 * crt_nrb(np); }

const CrtConst *crt_constants(int K)
{
    static std::once_flag once[5];
    static CrtConst table[5];
    static bool ok[5];
    if (K < 256 || K > 1024 || K % 256 != 0) return nullptr;
    const int i = K / 256;
    std::call_once(once[i], [&] { ok[i] = crt_setup(K, table[i]); });
    return ok[i] ? &table[i] : nullptr;
}

size_t crt_residue_bytes(int np, int K, int batch) { return crt_theta_bytes(np, K) * batch; }

void launch_crt_split(const double *A, int lda, size_t bstride, int np, int pe, int kc0, int K,
                      int batch, const CrtConst &cc, int8_t *sl, int32_t *ex, hipStream_t s,
                      const uint8_t *mask)
{
    const int m = np - pe;
    if (m <= 0) return;
    ProfScope ps(K_CRT_SPLIT, 0.0, (8.0 * K + (double)CRT_NMOD * K + 4.0) * m * batch, s);
    dim3 grid(m / 16, batch);
    const size_t sl_stride = crt_theta_bytes(np, K);
    const int nrb = crt_nrb(m);
    switch (K / 256) {
    case 1: crt_split_kernel<1><<<grid, 256, 0, s>>>(A, lda, bstride, pe, kc0, nrb, cc, sl, sl_stride, ex, np, mask); break;
    case 2: crt_split_kernel<2><<<grid, 256, 0, s>>>(A, lda, bstride, pe, kc0, nrb, cc, sl, sl_stride, ex, np, mask); break;
    case 3: crt_split_kernel<3><<<grid, 256, 0, s>>>(A, lda, bstride, pe, kc0, nrb, cc, sl, sl_stride, ex, np, mask); break;
    default: crt_split_kernel<4><<<grid, 256, 0, s>>>(A, lda, bstride, pe, kc0, nrb, cc, sl, sl_stride, ex, np, mask); break;
    }
}

}  // namespace gpk

namespace gpk {

void launch_syrk_update_crt(double *A, int lda, size_t bstride, int np, int pe, int cs, int ce,
                            int K, int batch, const CrtConst &cc, const int8_t *sl,
                            const int32_t *ex, hipStream_t s, const uint8_t *mask)
{
    if (ce <= cs || cs >= np) return;
    const int m = np - pe;
    const int NT = (m + 127) / 128;
    const int jt0 = (cs - pe) / 128, NC = (ce - cs + 127) / 128;
    int ntiles = 0;
    for (int jt = jt0; jt < jt0 + NC; ++jt) ntiles += NT - jt;
    if ((K / 64) % CRT_CPB != 0) return;   // K is a multiple of 256
    const double entries = (double)(ce - cs) * (np - cs) - 0.5 * (double)(ce - cs) * (ce - cs - 1);
    ProfScope ps(K_SYRK_UPDATE_CRT, 2.0 * K * entries * batch,
                 (16.0 * entries + (double)CRT_NMOD * K * (np - cs)) * batch, s);
    const long W = (long)ntiles * batch;
    const long per = (W + NXCD_CRT - 1) / NXCD_CRT;
    syrk_update_crt_kernel<CRT_NST, CRT_CPB><<<(unsigned)(per * NXCD_CRT), CRT_THREADS, 0, s>>>(
        A, lda, bstride, pe, m, ce - pe, jt0, jt0 + NC, NT, ntiles, batch, K / 64, crt_nrb(m), cc,
        sl, crt_theta_bytes(np, K), ex, np, mask);
}

}  // namespace gpk
