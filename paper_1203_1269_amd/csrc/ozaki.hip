// Matched-accuracy trailing update on INT8 MFMA (GP_MIXED).
//
// The rank-K update C -= P P^T of the blocked Cholesky (P: the m x K block of
// the factor below a finished outer panel) is computed by an error-free
// splitting of P in the style of Ozaki, Ogita, Oishi and Rump (Numer.
// Algorithms 59, 2012):
//   * every row i of P gets a power-of-two scale 2^e_i >= max_k |P_ik|, so
//     r_ik = P_ik 2^-e_i lies in (-1, 1);
//   * r_ik is cut into OZ_S signed 7-bit digits by repeated truncation,
//     r = sum_t d_t 2^(-7(t+1)) + rest, |d_t| <= 127, |rest| < 2^(-7 OZ_S);
//     every step (scale by 128, take the integer part, keep the remainder)
//     is exact in FP64;
//   * (P P^T)_ij = 2^(e_i + e_j) sum_{t,u} 2^(-7(t+u+2)) (D_t D_u^T)_ij, and
//     each digit product D_t D_u^T is an INT8 matrix product accumulated
//     exactly in INT32 (|sum| <= K 127^2 per pair);
//   * only the pairs with t + u < OZ_S are formed (the dropped ones are below
//     2^(-7 OZ_S) relative to the row scales); pairs with the same t + u share
//     one INT32 accumulator (at most OZ_S K 127^2 < 2^31 for K <= 2048), and the
//     levels are combined in FP64, smallest first, then scaled and subtracted
//     from the FP64 trailing matrix.
// With 8 digits the update carries about 56 significant bits relative to the
// row scales, as many as the FP64 update: -2logL agrees with the FP64 path
// to far below 1e-8 relative (a CPU emulation of the blocked factorisation
// gives 1e-10 or less where 7 digits leave up to 6e-9 on ill-conditioned R).
//
// v_mfma_i32_16x16x64_i8 layout (measured on gfx950): A[i][k] in lane
// i + 16 (k / 16), byte k % 16 of the lane's 16 bytes; B[k][j] in lane
// j + 16 (k / 16), byte k % 16; D[i][j] in lane j + 16 (i / 4), element i % 4.
// The digits are stored in exactly that fragment order, so every fragment is
// one contiguous 1 KiB load of 16 bytes per lane.  The product is formed as
// D = P_J P_I^T (A operand = rows of the column block, B operand = rows of
// the row block), so each lane's accumulator elements map to one output row
// and four columns, and 16 consecutive lanes store 16 consecutive rows of
// one column of the column-major matrix.
#include "kernels.hpp"

namespace gpk {
namespace {

typedef int int4v __attribute__((ext_vector_type(4)));

constexpr int OZ_K = OZ_RANK;          // update rank handled (outer panel width)
constexpr int OZ_KC = OZ_K / 64;       // 64-deep k chunks per fragment row block
constexpr int OZ_CPW = OZ_KC / 4;      // chunks per wave in the split kernel
static_assert(OZ_KC % 4 == 0, "the split kernel gives each of its 4 waves whole chunks");
static_assert(OZ_S * OZ_K * 127 * 127 < 2147483647, "INT32 level accumulators overflow");
constexpr int NXCD_OZ = 8;

// 2^(-7 (g + 2)): weight of digit level g (exact)
__host__ __device__ constexpr double level_weight(int g)
{
    double w = 1.0 / 16384.0;
    for (int q = 0; q < g; ++q) w *= 1.0 / 128.0;
    return w;
}

// bytes of one theta's digits for one slice: np rows * K bytes
__host__ __device__ inline size_t slice_bytes(int np) { return (size_t)np * OZ_K; }

// Byte offset of the 1 KiB fragment (digit t, 16-row block rb, 64-deep k
// chunk kc) within one theta's digits (nrb = np / 16 row blocks): chunk-major,
// then row block, then digit, so the digits of consecutive row blocks of one
// chunk are one contiguous run (32 KiB for the 64 rows of a tile).
__host__ __device__ inline size_t frag_off(int t, int rb, int kc, int nrb)
{
    return (((size_t)kc * nrb + rb) * OZ_S + t) * 1024;
}

// One workgroup per 16 rows of P: wave w covers k chunks w, w + 4, ...; lane l
// row l % 16 and k bytes 16 (l / 16) .. + 15 of each of its chunks.
__global__ __launch_bounds__(256)
void ozaki_split_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int pe,
                        int kc0, int8_t *__restrict__ sl0, int32_t *__restrict__ ex0,
                        const uint8_t *__restrict__ mask)
{
    const int b = blockIdx.y;
    if (mask && !mask[b]) return;   // uniform over the workgroup
    __shared__ double wmax[4][16];
    const int rb = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = 16 * rb + (lane & 15);           // row of P (0 .. m-1)
    const double *A = A0 + (size_t)b * bstride + (size_t)(pe + row) +
                      (size_t)(kc0 + 64 * wave + 16 * (lane >> 4)) * lda;
    double v[OZ_CPW][16];
    double m = 0.0;
#pragma unroll
    for (int h = 0; h < OZ_CPW; ++h)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            v[h][q] = A[(size_t)(256 * h + q) * lda];   // chunk wave + 4 h
            m = fmax(m, fabs(v[h][q]));
        }
    m = fmax(m, __shfl_xor(m, 16, 64));
    m = fmax(m, __shfl_xor(m, 32, 64));
    if (lane < 16) wmax[wave][lane] = m;
    __syncthreads();
    m = fmax(fmax(wmax[0][lane & 15], wmax[1][lane & 15]),
             fmax(wmax[2][lane & 15], wmax[3][lane & 15]));
    int e;
    (void)frexp(m, &e);   // m < 2^e (e = 0 for an all-zero row)
    int32_t *ex = ex0 + (size_t)b * np;
    if (wave == 0 && lane < 16) ex[row] = e;

    int8_t *sl = sl0 + (size_t)b * OZ_S * slice_bytes(np) + (size_t)lane * 16;
#pragma unroll
    for (int h = 0; h < OZ_CPW; ++h) {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[h][q] = ldexp(v[h][q], -e);   // |v| < 1, exact
#pragma unroll
        for (int t = 0; t < OZ_S; ++t) {
            int4v w;
#pragma unroll
            for (int word = 0; word < 4; ++word) {
                uint32_t packed = 0;
#pragma unroll
                for (int byte = 0; byte < 4; ++byte) {
                    const int q = 4 * word + byte;
                    const double x = v[h][q] * 128.0;
                    const double dg = trunc(x);      // |dg| <= 127
                    v[h][q] = x - dg;                // exact
                    packed |= ((uint32_t)(int)dg & 0xffu) << (8 * byte);
                }
                w[word] = (int)packed;
            }
            *(int4v *)(sl + frag_off(t, rb, wave + 4 * h, np / 16)) = w;
        }
    }
}

// 64 x 64 lower tiles of the m x m trailing matrix in tile columns
// jt0 .. (rows from the column's diagonal tile down), four waves of 32 x 32.
__global__ __launch_bounds__(256, 1)
void syrk_update_i8_kernel(double *__restrict__ A0, int lda, size_t bstride, int np, int pe,
                           int NT, int jt0, int ntiles, int batch,
                           const int8_t *__restrict__ sl0,
                           const int32_t *__restrict__ ex0, const uint8_t *__restrict__ mask)
{
    const int W = ntiles * batch;
    const int per = (W + NXCD_OZ - 1) / NXCD_OZ;
    const int bid = blockIdx.x;
    const int work = (bid % NXCD_OZ) * per + bid / NXCD_OZ;
    if (work >= W) return;
    const int b = work / ntiles;
    if (mask && !mask[b]) return;
    int t = work - b * ntiles;
    int jt = jt0;
    while (t >= NT - jt) { t -= NT - jt; ++jt; }
    const int it = jt + t;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rI = 64 * it + 32 * (wave >> 1);   // local row of the wave's block
    const int rJ = 64 * jt + 32 * (wave & 1);    // local column
    if (rI < rJ) return;                         // strictly upper: nothing to do; no barriers

    const int8_t *sl = sl0 + (size_t)b * OZ_S * slice_bytes(np);
    const int8_t *fI = sl + (size_t)lane * 16;
    const int8_t *fJ = sl + (size_t)lane * 16;

    int4v acc[OZ_S][2][2];
#pragma unroll
    for (int g = 0; g < OZ_S; ++g)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc[g][q][p] = (int4v){0, 0, 0, 0};

    // two fragment buffers: the loads of chunk kc + 1 are issued before the
    // MFMAs of chunk kc, so their latency hides behind a whole chunk of work
    int4v fa[2][OZ_S][2], fb[2][OZ_S][2];
    auto load_chunk = [&](int kc, int buf) {
#pragma unroll
        for (int sl_t = 0; sl_t < OZ_S; ++sl_t)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                fa[buf][sl_t][q] =
                    *(const int4v *)(fJ + frag_off(sl_t, rJ / 16 + q, kc, np / 16));
                fb[buf][sl_t][q] =
                    *(const int4v *)(fI + frag_off(sl_t, rI / 16 + q, kc, np / 16));
            }
    };
    load_chunk(0, 0);
    // D[a][b] of block (q, p): column rJ + 16 q + 4 (lane / 16) + e, row rI + 16 p + lane % 16.
    // The exponents and the C values are fetched while the last chunk's MFMAs
    // run (the second fragment buffer is free then).
    const int32_t *ex = ex0 + (size_t)b * np;
    double *A = A0 + (size_t)b * bstride;
    int eI[2], eJ[2][4];
    double cv[2][2][4];
#pragma unroll
    for (int kc = 0; kc < OZ_KC; ++kc) {
        const int cur = kc & 1;
        if (kc + 1 < OZ_KC) {
            load_chunk(kc + 1, cur ^ 1);
        } else {
#pragma unroll
            for (int p = 0; p < 2; ++p) eI[p] = ex[rI + 16 * p + (lane & 15)];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) eJ[q][e] = ex[rJ + 16 * q + 4 * (lane >> 4) + e];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        cv[q][p][e] = A[(size_t)(pe + rI + 16 * p + (lane & 15)) +
                                        (size_t)(pe + rJ + 16 * q + 4 * (lane >> 4) + e) * lda];
        }
        // keep the scheduler from sinking those loads towards their use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < OZ_S; ++u)
#pragma unroll
            for (int t = 0; t < OZ_S - u; ++t)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int p = 0; p < 2; ++p)
                        acc[t + u][q][p] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            fa[cur][t][q], fb[cur][u][p], acc[t + u][q][p], 0, 0, 0);
    }

#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double v = 0.0;
#pragma unroll
                for (int g = OZ_S - 1; g >= 0; --g)
                    v = fma((double)acc[g][q][p][e], level_weight(g), v);
                const int gi = pe + rI + 16 * p + (lane & 15);
                const int gj = pe + rJ + 16 * q + 4 * (lane >> 4) + e;
                A[(size_t)gi + (size_t)gj * lda] = cv[q][p][e] - ldexp(v, eI[p] + eJ[q][e]);
            }
}

}  // namespace

size_t ozaki_slices_bytes(int np, int batch) { return (size_t)OZ_S * slice_bytes(np) * batch; }

bool ozaki_handles(int np, int pe, int K) { return K == OZ_K && (np - pe) % 64 == 0; }

void launch_ozaki_split(const double *A, int lda, size_t bstride, int np, int pe, int kc0, int K,
                        int batch, int8_t *sl, int32_t *ex, hipStream_t s, const uint8_t *mask)
{
    const int m = np - pe;
    if (m <= 0) return;
    ProfScope ps(K_OZAKI_SPLIT, 0.0, (8.0 * K + (double)OZ_S * K + 4.0) * m * batch, s);
    dim3 grid(m / 16, batch);
    ozaki_split_kernel<<<grid, 256, 0, s>>>(A, lda, bstride, np, pe, kc0, sl, ex, mask);
}

void launch_syrk_update_i8(double *A, int lda, size_t bstride, int np, int pe, int cs, int ce,
                           int K, int batch, const int8_t *sl, const int32_t *ex, hipStream_t s,
                           const uint8_t *mask)
{
    if (ce <= cs || cs >= np) return;
    const int NT = (np - pe) / 64;
    const int jt0 = (cs - pe) / 64, NC = (ce - cs) / 64;
    int ntiles = 0;
    for (int jt = jt0; jt < jt0 + NC; ++jt) ntiles += NT - jt;
    const double entries = (double)(ce - cs) * (np - cs) - 0.5 * (double)(ce - cs) * (ce - cs - 1);
    ProfScope ps(K_SYRK_UPDATE_I8, 2.0 * K * entries * batch,
                 (16.0 * entries + (double)OZ_S * K * (np - cs)) * batch, s);
    const long W = (long)ntiles * batch;
    const long per = (W + NXCD_OZ - 1) / NXCD_OZ;
    syrk_update_i8_kernel<<<(unsigned)(per * NXCD_OZ), 256, 0, s>>>(
        A, lda, bstride, np, pe, NT, jt0, ntiles, batch, sl, ex, mask);
}

}  // namespace gpk
