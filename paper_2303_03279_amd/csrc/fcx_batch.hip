// Batch (window recompute) kernels: the network of K cached trials in one
// pass, with the Gram-type sums on the matrix cores.
//
//   k_psd_batch     P[b][i] = sum over the K trials of the per-trial power
//   k_pair_batch    per 32x32 quarter tile and bin:
//                     S = sum_k X_i conj(X_j)        MFMA (complex Gram as
//                     U = sum_k u_i conj(u_j)         real GEMMs; L = 1 for U)
//                   and per pair on the vector units, over the trials:
//                     G = sum sign(Im), A = sum |Im|, Q = sum Im^2
//                   then the seven metrics and their band mean
//   k_cor_batch     per 128x128 tile: sum over trials of the per-trial Pearson r
//                   as an LDS-staged MFMA GEMM over the z-scored samples
//
// The Gram operands run in the session's precision: FP32
// (v_mfma_f32_16x16x4f32), BF16 (v_mfma_f32_16x16x32_bf16, operands rounded
// to nearest even) or split BF16x3 (x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi), all with FP32
// accumulation.  Multitaper trials enter the CSD Gram as separate columns
// weighted by sqrt(lambda_l / sum lambda).
#include "fcx_device.h"

namespace fcx {

constexpr int BT_THREADS = 256;
constexpr int BT_CC = 32;           // contraction columns (trial x taper) staged per chunk
constexpr int BT_LD = BT_CC + 1;    // LDS row stride in float2 (spreads banks)

// ---------------------------------------------------------------- operands
// One chunk of BT_CC columns of the complex Gram for a 16x16 block:
// re += Re_a Re_b + Im_a Im_b, im += Im_a Re_b - Re_a Im_b.
// FP32: X is LDS [64 nodes][BT_LD] float2; the BF16 forms read planes (below).
// arow / bcol: this lane's A row node and B column node; lg = lane >> 4.
template <int PREC> struct Gram;

template <> struct Gram<FCX_GRAM_FP32_ID> {
    __device__ static void chunk(const float2 *X, int arow, int bcol, int lg, floatx4 &re, floatx4 &im)
    {
#pragma unroll
        for (int st = 0; st < BT_CC / 4; ++st) {
            const float2 a = X[arow * BT_LD + 4 * st + lg];
            const float2 b = X[bcol * BT_LD + 4 * st + lg];
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, b.y, im, 0, 0, 0);
        }
    }
};

// BF16 forms: the operands were rounded once, as they entered LDS, into
// planes of rows of BT_LDH values: plane 0 Re hi, 1 Im hi, 2 Re lo, 3 Im lo
// (lo = bf16(x - hi), BF16x3 only).  Lane group lg reads the 8 columns
// 8lg..8lg+7 of its row as one 16-byte load; -Re is Re with the sign bits
// flipped (rounding to nearest commutes with negation).
constexpr int BT_LDH = BT_CC + 8;   // 80-byte rows: the 16-byte lane reads hit distinct banks
constexpr int BT_PLANE = 64 * BT_LDH;

__device__ __forceinline__ bf16x8 bf_row(const __bf16 *P, int plane, int node, int lg)
{
    return *(const bf16x8 *)(P + plane * BT_PLANE + node * BT_LDH + 8 * lg);
}

__device__ __forceinline__ bf16x8 bf_neg(bf16x8 v)
{
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(bf16x8, __builtin_bit_cast(u32x4, v) ^ 0x80008000u);
}

template <> struct Gram<FCX_GRAM_BF16_ID> {
    __device__ static void chunk(const __bf16 *P, int arow, int bcol, int lg, floatx4 &re, floatx4 &im)
    {
        const bf16x8 ar = bf_row(P, 0, arow, lg), ai = bf_row(P, 1, arow, lg);
        const bf16x8 br = bf_row(P, 0, bcol, lg), bi = bf_row(P, 1, bcol, lg);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf_neg(ar), bi, im, 0, 0, 0);
    }
};

template <> struct Gram<FCX_GRAM_BF16X3_ID> {
    __device__ static void chunk(const __bf16 *P, int arow, int bcol, int lg, floatx4 &re, floatx4 &im)
    {
        const bf16x8 arh = bf_row(P, 0, arow, lg), aih = bf_row(P, 1, arow, lg);
        const bf16x8 arl = bf_row(P, 2, arow, lg), ail = bf_row(P, 3, arow, lg);
        const bf16x8 brh = bf_row(P, 0, bcol, lg), bih = bf_row(P, 1, bcol, lg);
        const bf16x8 brl = bf_row(P, 2, bcol, lg), bil = bf_row(P, 3, bcol, lg);
        const bf16x8 anh = bf_neg(arh), anl = bf_neg(arl);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brh, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brl, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, brh, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bih, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bil, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bih, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brh, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brl, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, brh, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bih, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anh, bil, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(anl, bih, im, 0, 0, 0);
    }
};

// the planes of one staged value
template <int PREC> __device__ __forceinline__ void bf_stage(__bf16 *P, int node, int col, float2 v)
{
    const __bf16 hr = (__bf16)v.x, hi = (__bf16)v.y;
    P[0 * BT_PLANE + node * BT_LDH + col] = hr;
    P[1 * BT_PLANE + node * BT_LDH + col] = hi;
    if (PREC == FCX_GRAM_BF16X3_ID) {
        P[2 * BT_PLANE + node * BT_LDH + col] = (__bf16)(v.x - (float)hr);
        P[3 * BT_PLANE + node * BT_LDH + col] = (__bf16)(v.y - (float)hi);
    }
}

// ------------------------------------------------------------- power sums
// 64 (bin, node) entries per workgroup; its four wavefronts take every fourth
// trial and their partial sums are added in wavefront order
__global__ __launch_bounds__(256) void k_psd_batch(SessDev<float> s, int K)
{
    __shared__ double part[3][64];
    if (s.ctl->bad) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const bool live = e < s.B * s.N;
    const int b = live ? e / s.N : 0, i = live ? e % s.N : 0;
    const float2 *ring = (const float2 *)s.ring;
    double p = 0.0;
    if (live)
        for (int t = w; t < K; t += 4)
            for (int l = 0; l < s.L; ++l) {
                const float2 v = ring[(((size_t)t * s.B + b) * s.L + l) * s.N + i];
                p += s.lamw[l] * ((double)v.x * v.x + (double)v.y * v.y);
            }
    if (w) part[w - 1][lane] = p;
    __syncthreads();
    if (w == 0 && live) s.psd[e] = ((p + part[0][lane]) + part[1][lane]) + part[2][lane];
}

// --------------------------------------------------------- pairs, one taper
// One 64x64 pair tile per workgroup of 8 wavefronts.  Wavefront w owns 16
// tile rows (block 16(w >> 1)) and the columns 32(w & 1) .. +31 as two 16x16
// MFMA blocks.  The MFMA's row r feeds from tile row pi(r) = (r >> 2) +
// 4 (r & 3) of the block, so lane (lr = lane & 15, lg = lane >> 4), which
// holds the accumulator rows 4lg + k of column lr, holds the pairs of tile
// rows lg + 4k (k < 4) and columns 16c + lr (c < 2): 8 pairs, whose vector
// sums it also keeps, so the epilogue of a bin finds every sum of a pair in
// one lane.  (The permutation makes the four lane groups read four
// consecutive rows: their 16-byte LDS reads fall in distinct banks.)
//
// Per trial the vector units form v = Im(X_i conj X_j) in FP64 from the FP32
// spectra: both products are exact in FP64, so v is the correctly rounded
// value of the exact difference.  Its sign is therefore exact (an exact zero
// gives +0: the first product enters as fma(-a, b, +0), which is never -0),
// and v, |v| and v^2 are summed in FP64, so Im S, A and Q carry no FP32
// growth and no Gram rounding.  The matrix cores compute Re S and the unit
// phasor Gram (and Im S too when no vector sums are asked for).
//
// A chunk of PB_CC trials of the 64 row and 64 column nodes is staged in LDS
// (rows in FP64, columns in FP32, unit phasors, BF16 planes for the BF16
// Grams) while the next chunk is already loaded into registers.
constexpr int PB_THREADS = 512;
constexpr int PB_CC = 32;             // trials per staged chunk (one 16x16x32 BF16 step)
constexpr int PB_LD = PB_CC + 1;      // LDS row stride of float2 / double2 rows
constexpr int PB_PER = 128 * PB_CC / PB_THREADS;   // staged values per thread and chunk
constexpr int PB_LDH = PB_CC + 8;     // BF16 plane rows (80 bytes)
constexpr int PB_PLANE = 128 * PB_LDH;

__device__ __forceinline__ int pb_perm(int r) { return (r >> 2) + 4 * (r & 3); }

template <int PREC> __device__ __forceinline__ void pb_stage(__bf16 *P, int node, int col, float2 v)
{
    const __bf16 hr = (__bf16)v.x, hi = (__bf16)v.y;
    P[0 * PB_PLANE + node * PB_LDH + col] = hr;
    P[1 * PB_PLANE + node * PB_LDH + col] = hi;
    if (PREC == FCX_GRAM_BF16X3_ID) {
        P[2 * PB_PLANE + node * PB_LDH + col] = (__bf16)(v.x - (float)hr);
        P[3 * PB_PLANE + node * PB_LDH + col] = (__bf16)(v.y - (float)hi);
    }
}

__device__ __forceinline__ bf16x8 pb_row(const __bf16 *P, int plane, int node, int lg)
{
    return *(const bf16x8 *)(P + plane * PB_PLANE + node * PB_LDH + 8 * lg);
}

// unit phasor X / |X| (0 for X = 0): FP32 where |X|^2 is safely inside the
// normal range, otherwise with the magnitude formed in FP64
__device__ __forceinline__ float2 pb_phasor(float2 x)
{
    const float m2 = __builtin_fmaf(x.x, x.x, x.y * x.y);
    if (m2 >= 0x1p-100f && m2 <= 0x1p100f) {
        const float r = __builtin_amdgcn_rsqf(m2);
        return make_float2(x.x * r, x.y * r);
    }
    const double d2 = (double)x.x * x.x + (double)x.y * x.y;
    const double r = d2 > 0.0 ? __builtin_amdgcn_rsq(d2) : 0.0;
    return make_float2((float)(x.x * r), (float)(x.y * r));
}

// Complex Gram of one 32-trial chunk for the lane's two 16x16 blocks: Re S
// always; Im S when IM.  FP32: A operand from the FP64 rows Ar (or FP32 rows
// when Ar is null), B operand from the FP32 columns; BF16: the planes.
template <int PREC, bool IM>
__device__ __forceinline__ void pb_gram(const double2 *Ar, const float2 *Af, const float2 *Bc, const __bf16 *Ph,
                                        int arow, int bcol0, int hrow, int hcol0, int lg, floatx4 (&re)[2],
                                        floatx4 (&im)[2])
{
    if constexpr (PREC == FCX_GRAM_FP32_ID) {
#pragma unroll
        for (int st = 0; st < PB_CC / 4; ++st) {
            float2 a;
            if (Ar) {
                const double2 ad = Ar[arow * PB_LD + 4 * st + lg];
                a = make_float2((float)ad.x, (float)ad.y);
            } else {
                a = Af[arow * PB_LD + 4 * st + lg];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float2 b = Bc[(bcol0 + 16 * c) * PB_LD + 4 * st + lg];
                re[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, re[c], 0, 0, 0);
                re[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, re[c], 0, 0, 0);
                if constexpr (IM) {
                    im[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, im[c], 0, 0, 0);
                    im[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, b.y, im[c], 0, 0, 0);
                }
            }
        }
    } else {
        constexpr bool X3 = PREC == FCX_GRAM_BF16X3_ID;
        const bf16x8 arh = pb_row(Ph, 0, hrow, lg), aih = pb_row(Ph, 1, hrow, lg);
        bf16x8 arl = arh, ail = aih;
        if constexpr (X3) {
            arl = pb_row(Ph, 2, hrow, lg);
            ail = pb_row(Ph, 3, hrow, lg);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int bn = hcol0 + 16 * c;
            const bf16x8 brh = pb_row(Ph, 0, bn, lg), bih = pb_row(Ph, 1, bn, lg);
#define FCX_MF(acc, a, b) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0)
            FCX_MF(re[c], arh, brh);
            FCX_MF(re[c], aih, bih);
            if constexpr (IM) {
                FCX_MF(im[c], aih, brh);
                FCX_MF(im[c], bf_neg(arh), bih);
            }
            if constexpr (X3) {
                const bf16x8 brl = pb_row(Ph, 2, bn, lg), bil = pb_row(Ph, 3, bn, lg);
                FCX_MF(re[c], arh, brl);
                FCX_MF(re[c], arl, brh);
                FCX_MF(re[c], aih, bil);
                FCX_MF(re[c], ail, bih);
                if constexpr (IM) {
                    FCX_MF(im[c], aih, brl);
                    FCX_MF(im[c], ail, brh);
                    FCX_MF(im[c], bf_neg(arh), bil);
                    FCX_MF(im[c], bf_neg(arl), bih);
                }
            }
#undef FCX_MF
        }
    }
}

template <int PREC, bool VS>
__global__ __launch_bounds__(PB_THREADS) void k_pair_batch1(SessDev<float> s, int K)
{
    constexpr bool BFP = PREC != FCX_GRAM_FP32_ID;
    constexpr int NPL = PREC == FCX_GRAM_BF16X3_ID ? 4 : 2;
    constexpr bool XR = VS;                 // rows in FP64 (vector sums; FP32 Gram A operand)
    constexpr bool XF = !VS && !BFP;        // rows in FP32 (FP32 Gram without vector sums)
    constexpr bool XC = VS || !BFP;         // columns in FP32
    __shared__ double2 Xr[XR ? 64 * PB_LD : 1];
    __shared__ float2 Xf[XF ? 64 * PB_LD : 1];
    __shared__ float2 Xc[XC ? 64 * PB_LD : 1];
    __shared__ float2 Us[BFP ? 1 : 128 * PB_LD];       // FP32 unit phasors, rows then columns
    __shared__ __attribute__((aligned(16))) __bf16 Xh[BFP ? NPL * PB_PLANE : 8];
    __shared__ __attribute__((aligned(16))) __bf16 Uh[BFP ? NPL * PB_PLANE : 8];
    __shared__ double SR[128];                          // 1/sqrt(P) of the staged nodes
    if (s.ctl->bad) return;
    const int tile = xcd_item(blockIdx.x, gridDim.x);
    const int2 tt = s.tiles[tile];
    const int R0 = tt.x * TILE, C0 = tt.y * TILE;
    const int N = s.N, B = s.B;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int wr = w >> 1, wc = w & 1;
    const int arow = 16 * wr + pb_perm(lr);   // Gram A operand: the row node of MFMA row lr
    const int bcol0 = 32 * wc + lr;           // Gram B operand of block 0: a column node
    const int rbase = 16 * wr + lg;           // the lane's pair rows rbase + 4k (tile rows)
    const int cbase = 32 * wc + lr;           // the lane's pair columns cbase + 16c (tile columns)
    const uint32_t mm = s.metrics;
    const bool needU = mm & M_PLV;
    const float2 *ring = (const float2 *)s.ring;
    const int nch = (K + PB_CC - 1) / PB_CC, total = B * nch;
    const float invK = 1.0f / (float)K;
    const float invKm1 = K >= 2 ? 1.0f / (float)(K - 1) : 0.f;
    const float Kf = (float)K;

    // staged value v of this thread: node e & 127 (64 rows, then 64 columns),
    // trial column (e >> 7) of the chunk, e = tid + PB_THREADS v
    const int snode = tid & 127, scol = tid >> 7;
    const int gnode = snode < 64 ? R0 + snode : C0 + snode - 64;
    const bool nodeok = gnode < N;
    const int gn = nodeok ? gnode : 0;
    auto fetch = [&](int cc, float2 (&dst)[PB_PER]) {
        const int b = cc / nch, t0 = (cc - b * nch) * PB_CC + scol;
        const bool ok = cc < total && nodeok;
        const float2 *base = ring + (size_t)b * N + gn;
#pragma unroll
        for (int v = 0; v < PB_PER; ++v) {
            const int t = t0 + 4 * v;
            const bool live = ok && t < K;
            const float2 x = base[(size_t)(live ? t : 0) * B * N];
            dst[v] = live ? x : make_float2(0.f, 0.f);
        }
    };
    float2 pre[PB_PER];
    fetch(0, pre);

    float acc[8][7];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int m = 0; m < 7; ++m) acc[p][m] = 0.f;

    for (int b = 0; b < B; ++b) {
        floatx4 sre[2], sim[2], ure[2], uim[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) sre[c] = sim[c] = ure[c] = uim[c] = (floatx4){0.f, 0.f, 0.f, 0.f};
        int G[8];
        double Sv[8], Av[8], Qv[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            G[p] = 0;
            Sv[p] = Av[p] = Qv[p] = 0.0;
        }
        for (int ch = 0; ch < nch; ++ch) {
            const int cc = b * nch + ch;
            const int nk = min(PB_CC, K - ch * PB_CC);
            __syncthreads();   // the previous chunk's readers are done
#pragma unroll
            for (int v = 0; v < PB_PER; ++v) {
                const int col = scol + 4 * v;
                const float2 x = pre[v];
                if (snode < 64) {
                    if constexpr (XR) Xr[snode * PB_LD + col] = make_double2(x.x, x.y);
                    if constexpr (XF) Xf[snode * PB_LD + col] = x;
                } else {
                    if constexpr (XC) Xc[(snode - 64) * PB_LD + col] = x;
                }
                if constexpr (BFP) {
                    pb_stage<PREC>(Xh, snode, col, x);
                    if (needU) pb_stage<PREC>(Uh, snode, col, pb_phasor(x));
                } else {
                    if (needU) Us[snode * PB_LD + col] = pb_phasor(x);
                }
            }
            if (ch == 0 && tid < 128) {
                const int g = tid < 64 ? R0 + tid : C0 + tid - 64;
                double r = 0.0;
                if (g < N) {
                    const double p = s.psd[(size_t)b * N + g];
                    r = p > 0.0 ? rsqrt(p) : 0.0;
                }
                SR[tid] = r;
            }
            __syncthreads();
            fetch(cc + 1, pre);   // the next chunk is on its way while this one is computed

            // FP32 Gram with vector sums: its steps (4 trials each) are
            // interleaved with the vector sums of the same trials below, so
            // the matrix cores work while the vector units sum
            constexpr bool MIX = VS && PREC == FCX_GRAM_FP32_ID;
            if constexpr (!MIX) {
                pb_gram<PREC, !VS>(XR ? Xr : nullptr, Xf, Xc, Xh, arow, bcol0, arow, 64 + bcol0, lg, sre, sim);
                if (needU)
                    pb_gram<PREC, true>(nullptr, Us, Us + 64 * PB_LD, Uh, arow, bcol0, arow, 64 + bcol0, lg, ure,
                                        uim);
            }
            // one FP32 Gram step: trials 4 st + lg of the chunk (Re S, and the
            // unit-phasor Gram); steps past the chunk's trials would add zeros
            auto gram_step = [&](int st) {
                const double2 ad = Xr[arow * PB_LD + 4 * st + lg];
                const float2 a = make_float2((float)ad.x, (float)ad.y);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float2 bb = Xc[(bcol0 + 16 * c) * PB_LD + 4 * st + lg];
                    sre[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, sre[c], 0, 0, 0);
                    sre[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, sre[c], 0, 0, 0);
                }
                if (needU) {
                    const float2 ua = Us[arow * PB_LD + 4 * st + lg];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const float2 ub = Us[(64 + bcol0 + 16 * c) * PB_LD + 4 * st + lg];
                        ure[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.x, ub.x, ure[c], 0, 0, 0);
                        ure[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.y, ub.y, ure[c], 0, 0, 0);
                        uim[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ua.y, ub.x, uim[c], 0, 0, 0);
                        uim[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ua.x, ub.y, uim[c], 0, 0, 0);
                    }
                }
            };
            if constexpr (VS) {
                // trial t's operands are loaded while trial t - 1 is summed;
                // columns past the trials are 0 and add nothing, and the pad
                // column PB_CC is loaded but never summed
                const double2 *xrp = Xr + rbase * PB_LD;
                const float2 *ycp = Xc + cbase * PB_LD;
                auto ldt = [&](int t, double2 (&xr)[4], float2 (&yc)[2]) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) xr[k] = xrp[4 * k * PB_LD + t];
#pragma unroll
                    for (int c = 0; c < 2; ++c) yc[c] = ycp[16 * c * PB_LD + t];
                };
                auto sum_t = [&](const double2 (&xr)[4], const float2 (&yc)[2]) {
                    const double jx[2] = {yc[0].x, yc[1].x}, jy[2] = {yc[0].y, yc[1].y};
#pragma unroll
                    for (int k = 0; k < 4; ++k)
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const double v = __builtin_fma(xr[k].y, jx[c], __builtin_fma(-xr[k].x, jy[c], 0.0));
                            const int p = 2 * k + c;
                            G[p] += sign_of_f64(v);
                            Av[p] = Av[p] + fabs(v);
                            Qv[p] = __builtin_fma(v, v, Qv[p]);
                            Sv[p] = Sv[p] + v;
                        }
                };
                double2 ra[4], rb[4];
                float2 ca[2], cb[2];
                ldt(0, ra, ca);
                if constexpr (MIX) {
                    for (int t = 0; t < nk; t += 4) {
                        gram_step(t >> 2);
                        ldt(t + 1, rb, cb);
                        sum_t(ra, ca);
                        ldt(t + 2, ra, ca);
                        sum_t(rb, cb);
                        ldt(t + 3, rb, cb);
                        sum_t(ra, ca);
                        ldt(min(t + 4, PB_CC), ra, ca);
                        sum_t(rb, cb);
                    }
                } else {
                    for (int t = 0; t < nk; t += 2) {
                        ldt(t + 1, rb, cb);
                        sum_t(ra, ca);
                        ldt(min(t + 2, PB_CC), ra, ca);
                        sum_t(rb, cb);
                    }
                }
            }
        }
        // metrics of this bin for the lane's pairs, into the band means
        // (computed for every lane; only pairs i < j < N are stored)
        double srr[4], src[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) srr[k] = SR[rbase + 4 * k];
#pragma unroll
        for (int c = 0; c < 2; ++c) src[c] = SR[64 + cbase + 16 * c];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int p = 2 * k + c;
                const double Sr = sre[c][k];
                const double Si = VS ? Sv[p] : (double)sim[c][k];
                const double srij = srr[k] * src[c];
                if (mm & M_COH) acc[p][0] += sqrt_ratio<float>((Sr * Sr + Si * Si) * srij * srij);
                if (mm & M_IMCOH) acc[p][1] += (float)(Si * srij);
                if (mm & M_PLV) {
                    const float ur = ure[c][k], ui = uim[c][k];
                    acc[p][2] += __builtin_amdgcn_sqrtf(ur * ur + ui * ui) * invK;
                }
                if constexpr (VS) {
                    const float pli = (float)abs(G[p]) * invK;
                    if (mm & M_PLI) acc[p][3] += pli;
                    if (mm & M_USPLI) acc[p][5] += K >= 2 ? (Kf * pli * pli - 1.0f) * invKm1 : NAN;
                    if (mm & M_WPLI) acc[p][4] += Av[p] > 0.0 ? ratio_t<float>(fabs(Si), Av[p]) : 0.f;
                    if (mm & M_DSWPLI) {
                        const double dd = Av[p] * Av[p] - Qv[p];
                        acc[p][6] += K >= 2 ? (dd != 0.0 ? ratio_t<float>(Si * Si - Qv[p], dd) : 0.f) : NAN;
                    }
                }
            }
    }
    const size_t P = (size_t)N * (N - 1) / 2;
    const float invB = 1.0f / (float)B;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = R0 + rbase + 4 * k, j = C0 + cbase + 16 * c;
            if (!(i < j && j < N)) continue;
            const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
#pragma unroll
            for (int m = 0; m < 7; ++m)
                if (mm & (1u << m)) s.out[(size_t)m * P + idx] = acc[2 * k + c][m] * invB;
        }
}

// ------------------------------------------------------ pairs, several tapers
// Per 32x32 quarter tile and bin (4 wavefronts of one 16x16 block each): the
// Gram of Re S over (trial, taper) columns weighted by sqrt(lambda_l / sum
// lambda) on the matrix cores; per pair and trial on the vector units the
// taper-combined CSD c = sum_l w_l X_il conj(X_jl) with each taper's products
// exact in FP64 (so Im c of a zero-lag pair is an exact 0), its sign, |Im c|,
// (Im c)^2 and Im c summed in FP64, and the unit phasor of c for PLV.
// LT: the number of tapers when fixed at compile time (0: s.L at run time).
template <int PREC, int LT>
__global__ __launch_bounds__(BT_THREADS) void k_pair_batchL(SessDev<float> s, int K)
{
    constexpr bool BFP = PREC != FCX_GRAM_FP32_ID;
    constexpr int NPL = PREC == FCX_GRAM_BF16X3_ID ? 4 : 2;   // BF16 planes per operand
    __shared__ float2 Xs[64 * BT_LD];                         // FP32 values (Gram operands, column nodes)
    __shared__ __attribute__((aligned(16))) __bf16 Xh[BFP ? NPL * BT_PLANE : 8];
    if (s.ctl->bad) return;
    const int tile = blockIdx.x >> 2, qd = blockIdx.x & 3;
    const int2 tt = s.tiles[tile];
    const int R0 = tt.x * TILE + 32 * (qd >> 1), C0 = tt.y * TILE + 32 * (qd & 1);
    const int N = s.N, B = s.B, L = LT ? LT : s.L;
    if (R0 >= N || R0 >= min(C0 + 31, N - 1)) return;   // no pair i < j < N here
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int wr = w >> 1, wc = w & 1;
    const int arow = 16 * wr + lr;           // LDS node of this lane's A fragment
    const int bcol = 32 + 16 * wc + lr;      // LDS node of this lane's B fragment = its pairs' column
    const int j = C0 + 16 * wc + lr;
    // accumulator element k of this lane: row 4*lg+k of the wave's block
    int rows[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rows[k] = 16 * wr + 4 * lg + k;
    const uint32_t mm = s.metrics;
    const bool needU = mm & M_PLV;
    const int TPC = BT_CC / L;   // whole trials per chunk
    const int CC = TPC * L;
    const float2 *ring = (const float2 *)s.ring;
    const double Kd = (double)K;

    float acc[4][7];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 7; ++m) acc[k][m] = 0.f;

    for (int b = 0; b < B; ++b) {
        floatx4 sre = {0.f, 0.f, 0.f, 0.f}, sdum = sre;
        int G[4] = {0, 0, 0, 0};
        double A[4] = {0, 0, 0, 0}, Q[4] = {0, 0, 0, 0}, S[4] = {0, 0, 0, 0};
        double VUr[4] = {0, 0, 0, 0}, VUi[4] = {0, 0, 0, 0};
        for (int t0 = 0; t0 < K; t0 += TPC) {
            const int nk = min(TPC, K - t0);
            __syncthreads();
            // consecutive lanes take consecutive nodes of one column, so a
            // wavefront reads two contiguous runs of 32 nodes
            for (int e = threadIdx.x; e < 64 * BT_CC; e += BT_THREADS) {
                const int node = e & 63, col = e >> 6;
                const int t = col / L, l = col % L;
                const int g = node < 32 ? R0 + node : C0 + node - 32;
                float2 v = make_float2(0.f, 0.f);
                if (col < CC && t < nk && g < N) {
                    v = ring[(((size_t)(t0 + t) * B + b) * L + l) * N + g];
                    const float wl = (float)sqrt(s.lamw[l]);
                    v.x *= wl;
                    v.y *= wl;
                }
                Xs[node * BT_LD + col] = v;
                if constexpr (BFP) bf_stage<PREC>(Xh, node, col, v);
            }
            __syncthreads();
            if constexpr (BFP) {
                Gram<PREC>::chunk(Xh, arow, bcol, lg, sre, sdum);
            } else {
                Gram<PREC>::chunk(Xs, arow, bcol, lg, sre, sdum);
            }
            for (int t = 0; t < nk; ++t) {
                double cr[4] = {0.0, 0.0, 0.0, 0.0}, ci[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll(LT ? LT : 1)
                for (int l = 0; l < L; ++l) {
                    const float2 xj = Xs[bcol * BT_LD + t * L + l];
                    const double jx = xj.x, jy = xj.y;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float2 xf = Xs[rows[k] * BT_LD + t * L + l];
                        const double2 xi = make_double2(xf.x, xf.y);
                        // each taper's Im exact-rounded in FP64 (both products exact; the
                        // +0 keeps an exact zero positive), then summed over the tapers
                        ci[k] = ci[k] + __builtin_fma(xi.y, jx, __builtin_fma(-xi.x, jy, 0.0));
                        if (needU) cr[k] = __builtin_fma(xi.x, jx, __builtin_fma(xi.y, jy, cr[k]));
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    G[k] += sign_of_f64(ci[k]);
                    A[k] = A[k] + fabs(ci[k]);
                    Q[k] = __builtin_fma(ci[k], ci[k], Q[k]);
                    S[k] = S[k] + ci[k];
                    if (needU) {   // the unit phasor of the taper-combined CSD
                        const float2 u = pb_phasor(make_float2((float)cr[k], (float)ci[k]));
                        VUr[k] += (double)u.x;
                        VUi[k] += (double)u.y;
                    }
                }
            }
        }
        // metrics of this bin for the lane's pairs, into the band means
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = R0 + rows[k];
            if (!(i < j && j < N)) continue;
            const double Sr = sre[k], Si = S[k];
            const double pp = s.psd[(size_t)b * N + i] * s.psd[(size_t)b * N + j];
            if (mm & M_COH) acc[k][0] += pp > 0.0 ? (float)sqrt((Sr * Sr + Si * Si) / pp) : 0.f;
            if (mm & M_IMCOH) acc[k][1] += pp > 0.0 ? (float)(Si / sqrt(pp)) : 0.f;
            if (mm & M_PLV) acc[k][2] += (float)(sqrt(VUr[k] * VUr[k] + VUi[k] * VUi[k]) / Kd);
            const double pli = fabs((double)G[k]) / Kd;
            if (mm & M_PLI) acc[k][3] += (float)pli;
            if (mm & M_USPLI) acc[k][5] += K >= 2 ? (float)((Kd * pli * pli - 1.0) / (Kd - 1.0)) : NAN;
            if (mm & M_WPLI) acc[k][4] += A[k] > 0.0 ? ratio_t<float>(fabs(Si), A[k]) : 0.f;
            if (mm & M_DSWPLI) {
                const double dd = A[k] * A[k] - Q[k];
                acc[k][6] += K >= 2 ? (dd != 0.0 ? ratio_t<float>(Si * Si - Q[k], dd) : 0.f) : NAN;
            }
        }
    }
    const size_t P = (size_t)N * (N - 1) / 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = R0 + rows[k];
        if (!(i < j && j < N)) continue;
        const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
#pragma unroll
        for (int m = 0; m < 7; ++m)
            if (mm & (1u << m)) s.out[(size_t)m * P + idx] = acc[k][m] / (float)B;
    }
}

// ------------------------------------------------------------------ COR
// One 128x128 tile of pairs per workgroup; each wavefront owns a block of
// CR_WR x CR_WC MFMA blocks of 16x16.  For every trial the z-scored samples
// of the tile's 128 row and 128 column nodes stream through LDS CR_CH samples
// at a time, in two buffers, while the next chunks are already on their way
// into registers.  The BF16 forms round the samples (and, for BF16x3, their
// remainders) once, as they are written to LDS.  Inside 32 samples lane group
// lg supplies samples 8lg..8lg+7 (the contraction order is free), so an
// operand fragment is one or two 16-byte LDS reads.  Each trial's r is
// accumulated in FP32 by the MFMAs and added to an FP64 sum at the trial's
// end, so the window sum carries no FP32 growth across trials.  Tiles are
// numbered in bands of CR_BAND tile rows (column by column inside a band) and
// each XCD takes a contiguous run of those numbers, so the workgroups resident
// on one XCD share a few row and column strips in its L2.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int CR_T = 128;     // tile edge in nodes
#ifndef FCX_COR_CH
#define FCX_COR_CH 32
#endif
constexpr int CR_CH = FCX_COR_CH;  // samples per staged chunk (divides the padded trial length)
constexpr int CR_LD = CR_CH + 4;   // LDS row stride in floats: 16-byte lane reads hit distinct banks
constexpr int CR_LDH = CR_CH + 8;  // the same for rows of BF16
constexpr int CR_BAND = 4;
#ifndef FCX_COR_WR
#define FCX_COR_WR 2
#endif
#ifndef FCX_COR_WC
#define FCX_COR_WC 4
#endif
#ifndef FCX_COR_PF32
#define FCX_COR_PF32 1      // chunks in flight ahead of the FP32 MFMAs
#endif
#ifndef FCX_COR_PF16
#define FCX_COR_PF16 3      // and ahead of the (shorter) BF16 ones
#endif

// Tile (row, column), row <= column, of number lin in the band order.
__device__ __forceinline__ int2 cor_tile(int lin, int T)
{
    for (int r0 = 0; r0 < T; r0 += CR_BAND) {
        const int h = min(CR_BAND, T - r0);
        const int tri = h * (h + 1) / 2;
        const int cnt = tri + (T - r0 - h) * h;
        if (lin < cnt) {
            if (lin < tri) {  // the band's diagonal block: column r0 + q holds rows r0 .. r0 + q
                int q = 0;
                while ((q + 1) * (q + 2) / 2 <= lin) ++q;
                return make_int2(r0 + lin - q * (q + 1) / 2, r0 + q);
            }
            lin -= tri;
            return make_int2(r0 + lin % h, r0 + h + lin / h);
        }
        lin -= cnt;
    }
    return make_int2(0, 0);
}

__device__ __forceinline__ float cor_pick(float4 v, int e)
{
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// The BF16 form reads the samples already rounded to BF16 (s.zbf, by
// k_z_bf16, the rounding the other forms apply as they stage), so a chunk
// moves half the bytes; FP32 and BF16x3 read the FP32 samples.
template <int PREC, int WR, int WC, int PF>
__global__ __launch_bounds__(64 * (CR_T / (16 * WR)) * (CR_T / (16 * WC))) void k_cor_batch(SessDev<float> s, int K,
                                                                                  int G, double *scratch, int *count)
{
    constexpr bool PRE = PREC == FCX_GRAM_BF16_ID;
    constexpr int WAVES_C = CR_T / (16 * WC);
    constexpr int NT = 64 * (CR_T / (16 * WR)) * WAVES_C;
    constexpr int SPV = PRE ? 8 : 4;                  // samples per staged 16-byte vector
    constexpr int V4 = 2 * CR_T * (CR_CH / SPV) / NT;  // vectors staged per thread and chunk
    static_assert(V4 * NT == 2 * CR_T * (CR_CH / SPV), "staging must cover the chunk");
    // one buffer: FP32 rows of CR_LD floats, or BF16 rows of CR_LDH (hi, then for
    // BF16x3 a plane of lo parts)
    constexpr int ZBUF = PREC == FCX_GRAM_FP32_ID ? 2 * CR_T * CR_LD
                         : (PREC == FCX_GRAM_BF16_ID ? 1 : 2) * 2 * CR_T * CR_LDH / 2;
    __shared__ __attribute__((aligned(16))) float Z[2][ZBUF];
    __shared__ int last;
    if (s.ctl->bad) return;
    const int N = s.N, Mz = s.Mz;
    const int T = (N + CR_T - 1) / CR_T;
    const int n = T * (T + 1) / 2;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int wr = w / WAVES_C, wc = w % WAVES_C;
    const size_t P = (size_t)N * (N - 1) / 2;
    // G resident workgroups; workgroups on one XCD hold neighbouring places.
    // Whole tiles go out round by round while at least two rounds remain; the
    // last ns tiles (G <= ns < 2G) are cut as ns x K units (tile, trial) into
    // G equal runs, each of at least K units, so such a tile is shared by at
    // most two workgroups.  With n <= G every workgroup takes one whole tile.
    const int xcd = blockIdx.x & 7, gq = G >> 3, grem = G & 7;
    const int pos = xcd * gq + min(xcd, grem) + (int)(blockIdx.x >> 3);
    const int rounds = n > G ? n / G - 1 : 0, nd = rounds * G;
    const long long U = (long long)(n - nd) * K, us1 = U * (pos + 1) / G;
    long long u = U * pos / G;
    for (int seg = 0;; ++seg) {
        int lin, t0, t1;
        if (seg < rounds) {
            lin = seg * G + pos;
            t0 = 0;
            t1 = K;
        } else {
            if (u >= us1) break;
            const int l = (int)(u / K);
            t0 = (int)(u - (long long)l * K);
            t1 = (int)min((long long)K, t0 + (us1 - u));
            u += t1 - t0;
            lin = nd + l;
        }
        const int2 tt = cor_tile(lin, T);
        const int I0 = tt.x * CR_T, J0 = tt.y * CR_T;

        // staging: vector number e = tid + NT v of a chunk is node e / (CR_CH / SPV)
        // (the 128 row nodes, then the 128 column nodes), samples SPV (e % (CR_CH / SPV))
        // .. + SPV - 1; rows past N read node N - 1 and only feed outputs never written
        unsigned off[V4];
        int lds[V4];
#pragma unroll
        for (int v = 0; v < V4; ++v) {
            const int e = tid + NT * v, node = e / (CR_CH / SPV), q4 = e % (CR_CH / SPV);
            const int g = min(node < CR_T ? I0 + node : J0 + node - CR_T, N - 1);
            off[v] = (unsigned)g * (unsigned)Mz + (unsigned)(SPV * q4);
            lds[v] = node * (PREC == FCX_GRAM_FP32_ID ? CR_LD : CR_LDH) + SPV * q4;
        }
        const int nch = Mz / CR_CH, cbeg = t0 * nch, total = t1 * nch;
        const size_t trial = (size_t)N * Mz;
        // chunk cc = trial * nch + chunk within the trial; chunks past the
        // segment's last load that one again (never used)
        // (element offset of the chunk; elements are floats, or BF16 with PRE)
        auto chunk_at = [&](int cc) {
            cc = min(cc, total - 1);
            const int tq = cc / nch;
            return (size_t)tq * trial + (size_t)(cc - tq * nch) * CR_CH;
        };
        auto load_chunk = [&](int cc, floatx4 (&dst)[V4]) {
            const size_t b = chunk_at(cc);
#pragma unroll
            for (int v = 0; v < V4; ++v) {
                if constexpr (PRE)
                    dst[v] = *(const floatx4 *)((const __bf16 *)s.zbf + b + off[v]);
                else
                    dst[v] = *(const floatx4 *)(s.zring + b + off[v]);
            }
        };
        floatx4 pre[PF][V4];
#pragma unroll
        for (int p = 0; p < PF; ++p) load_chunk(cbeg + p, pre[p]);
        floatx4 acc[WR][WC];
        double R[WR][WC][4];
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
            for (int j = 0; j < WC; ++j) {
                acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < 4; ++k) R[i][j][k] = 0.0;
            }
        for (int c0 = cbeg; c0 < total; c0 += PF) {
#pragma unroll
            for (int p = 0; p < PF; ++p) {
                const int c = c0 + p;
                if (c >= total) break;
                float *Zb = Z[c & 1];
#pragma unroll
                for (int v = 0; v < V4; ++v) {
                    const floatx4 x = pre[p][v];
                    if (PREC == FCX_GRAM_FP32_ID) {
                        *(floatx4 *)(Zb + lds[v]) = x;
                    } else if (PRE) {  // 8 samples already in BF16
                        *(floatx4 *)((__bf16 *)Zb + lds[v]) = x;
                    } else {  // rounded once here, for every wavefront that reads it
                        __bf16 *Zh = (__bf16 *)Zb;
                        const bf16x4 h = {(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
                        *(bf16x4 *)(Zh + lds[v]) = h;
                        if (PREC == FCX_GRAM_BF16X3_ID)
                            *(bf16x4 *)(Zh + 2 * CR_T * CR_LDH + lds[v]) =
                                (bf16x4){(__bf16)(x[0] - (float)h[0]), (__bf16)(x[1] - (float)h[1]),
                                         (__bf16)(x[2] - (float)h[2]), (__bf16)(x[3] - (float)h[3])};
                    }
                }
                __syncthreads();
                load_chunk(c + PF, pre[p]);   // chunk c + PF into the registers just emptied
                __builtin_amdgcn_sched_barrier(0);  // the loads go out before the chunk's LDS reads and MFMAs
#pragma unroll
                for (int sub = 0; sub < CR_CH / 32; ++sub) {
                    const float *Ap = Zb + (16 * WR * wr + lr) * CR_LD + 32 * sub + 8 * lg;
                    const float *Bp = Zb + (CR_T + 16 * WC * wc + lr) * CR_LD + 32 * sub + 8 * lg;
                    if (PREC == FCX_GRAM_FP32_ID) {
#pragma unroll
                        for (int half = 0; half < 2; ++half) {
                            float4 a[WR], b[WC];
#pragma unroll
                            for (int i = 0; i < WR; ++i) a[i] = *(const float4 *)(Ap + 16 * i * CR_LD + 4 * half);
#pragma unroll
                            for (int j = 0; j < WC; ++j) b[j] = *(const float4 *)(Bp + 16 * j * CR_LD + 4 * half);
#pragma unroll
                            for (int e = 0; e < 4; ++e)
#pragma unroll
                                for (int i = 0; i < WR; ++i)
#pragma unroll
                                    for (int j = 0; j < WC; ++j)
                                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                            cor_pick(a[i], e), cor_pick(b[j], e), acc[i][j], 0, 0, 0);
                        }
                    } else {
                        const __bf16 *Zh = (const __bf16 *)Zb, *Zl = Zh + 2 * CR_T * CR_LDH;
                        const int ra = (16 * WR * wr + lr) * CR_LDH + 32 * sub + 8 * lg;
                        const int rb = (CR_T + 16 * WC * wc + lr) * CR_LDH + 32 * sub + 8 * lg;
                        bf16x8 ah[WR], bh[WC], al[WR], bl[WC];
#pragma unroll
                        for (int i = 0; i < WR; ++i) {
                            ah[i] = *(const bf16x8 *)(Zh + ra + 16 * i * CR_LDH);
                            if (PREC == FCX_GRAM_BF16X3_ID) al[i] = *(const bf16x8 *)(Zl + ra + 16 * i * CR_LDH);
                        }
#pragma unroll
                        for (int j = 0; j < WC; ++j) {
                            bh[j] = *(const bf16x8 *)(Zh + rb + 16 * j * CR_LDH);
                            if (PREC == FCX_GRAM_BF16X3_ID) bl[j] = *(const bf16x8 *)(Zl + rb + 16 * j * CR_LDH);
                        }
#pragma unroll
                        for (int i = 0; i < WR; ++i)
#pragma unroll
                            for (int j = 0; j < WC; ++j) {
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                                if (PREC == FCX_GRAM_BF16X3_ID) {
                                    acc[i][j] =
                                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                                    acc[i][j] =
                                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                                }
                            }
                    }
                }
                if ((c + 1) % nch == 0) {  // end of a trial: its r joins the FP64 window sum
#pragma unroll
                    for (int i = 0; i < WR; ++i)
#pragma unroll
                        for (int j = 0; j < WC; ++j) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) R[i][j][k] += (double)acc[i][j][k];
                            acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
                        }
                }
            }
        }
        const bool whole = t0 == 0 && t1 == K;
        if (!whole) {
            // a shared tile: both partial sums are added to the zeroed FP64
            // scratch (two addends, so the sum is the same in either order); the
            // workgroup that finishes second writes the tile
#pragma unroll
            for (int i = 0; i < WR; ++i)
#pragma unroll
                for (int j = 0; j < WC; ++j)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int r = I0 + 16 * WR * wr + 16 * i + 4 * lg + k, col = J0 + 16 * WC * wc + 16 * j + lr;
                        if (!(r < col && col < N)) continue;
                        const size_t idx = (size_t)r * (2 * (size_t)N - r - 1) / 2 + (size_t)(col - r - 1);
                        unsafeAtomicAdd(scratch + idx, R[i][j][k]);
                    }
            __threadfence();
            __syncthreads();
            if (tid == 0)
                last = __hip_atomic_fetch_add(count + lin, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1;
            __syncthreads();
        }
        if (whole || last) {
#pragma unroll
            for (int i = 0; i < WR; ++i)
#pragma unroll
                for (int j = 0; j < WC; ++j)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int r = I0 + 16 * WR * wr + 16 * i + 4 * lg + k, col = J0 + 16 * WC * wc + 16 * j + lr;
                        if (!(r < col && col < N)) continue;
                        const size_t idx = (size_t)r * (2 * (size_t)N - r - 1) / 2 + (size_t)(col - r - 1);
                        const double sum = whole ? R[i][j][k]
                                                 : __hip_atomic_load(scratch + idx, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
                        s.out[7 * P + idx] = (float)(sum / (double)K);
                    }
        }
        __syncthreads();  // LDS buffers and `last` are reused by the next segment
    }
}

// The K trials' z-scored samples (ring slots 0..K-1) rounded to BF16, four
// per thread and step, with the rounding the BF16 COR staging applies.
__global__ __launch_bounds__(256) void k_z_bf16(const float *__restrict__ z, __bf16 *__restrict__ zb, long long n4)
{
    for (long long q = blockIdx.x * 256LL + threadIdx.x; q < n4; q += (long long)gridDim.x * 256) {
        const floatx4 x = ((const floatx4 *)z)[q];
        ((bf16x4 *)zb)[q] = (bf16x4){(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
    }
}

// ------------------------------------------------------------------ launch
__global__ void k_set_pushed(DevCtl *c, long long pushed)
{
    if (threadIdx.x == 0) c->pushed = pushed;
}

__global__ void k_batch_commit(DevCtl *c, long long K)
{
    if (threadIdx.x == 0) {
        if (c->bad) {
            c->rejected = c->rejected + 1;
            c->pushed = 0;
        } else {
            c->pushed = K;
        }
        c->bad = 0;
    }
}

hipError_t launch_set_pushed(DevCtl *ctl, long long pushed, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_pushed, dim3(1), dim3(64), 0, st, ctl, pushed);
    return hipGetLastError();
}

hipError_t launch_batch_commit(DevCtl *ctl, long long K, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_commit, dim3(1), dim3(64), 0, st, ctl, K);
    return hipGetLastError();
}

hipError_t launch_psd_batch(const SessDev<float> &s, int K, hipStream_t st)
{
    hipLaunchKernelGGL(k_psd_batch, dim3((s.B * s.N + 63) / 64), dim3(256), 0, st, s, K);
    return hipGetLastError();
}

template <bool VS> static void launch_pair_batch1(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    const dim3 grid(s.ntiles), blk(PB_THREADS);
    switch (prec) {
    case FCX_GRAM_BF16_ID: hipLaunchKernelGGL((k_pair_batch1<FCX_GRAM_BF16_ID, VS>), grid, blk, 0, st, s, K); break;
    case FCX_GRAM_BF16X3_ID: hipLaunchKernelGGL((k_pair_batch1<FCX_GRAM_BF16X3_ID, VS>), grid, blk, 0, st, s, K); break;
    default: hipLaunchKernelGGL((k_pair_batch1<FCX_GRAM_FP32_ID, VS>), grid, blk, 0, st, s, K); break;
    }
}

hipError_t launch_pair_batch(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    if (s.L == 1) {
        // the sign, |Im|, Im^2 and Im sums run on the vector units only when a
        // metric needs them
        if (s.metrics & (M_PLI | M_WPLI | M_USPLI | M_DSWPLI))
            launch_pair_batch1<true>(s, K, prec, st);
        else
            launch_pair_batch1<false>(s, K, prec, st);
    } else {
        const dim3 grid(s.ntiles * 4), blk(BT_THREADS);
        // three tapers (the common DPSS choice) with the taper loop unrolled
        const bool l3 = s.L == 3;
        switch (prec) {
        case FCX_GRAM_BF16_ID:
            if (l3) hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_BF16_ID, 3>), grid, blk, 0, st, s, K);
            else hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_BF16_ID, 0>), grid, blk, 0, st, s, K);
            break;
        case FCX_GRAM_BF16X3_ID:
            if (l3) hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_BF16X3_ID, 3>), grid, blk, 0, st, s, K);
            else hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_BF16X3_ID, 0>), grid, blk, 0, st, s, K);
            break;
        default:
            if (l3) hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_FP32_ID, 3>), grid, blk, 0, st, s, K);
            else hipLaunchKernelGGL((k_pair_batchL<FCX_GRAM_FP32_ID, 0>), grid, blk, 0, st, s, K);
            break;
        }
    }
    return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_cor_batch(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    constexpr int WR = FCX_COR_WR, WC = FCX_COR_WC;
    constexpr int NT = 64 * (CR_T / (16 * WR)) * (CR_T / (16 * WC));
    const int T = (s.N + CR_T - 1) / CR_T;
    const int n = T * (T + 1) / 2;
    // one resident workgroup per compute unit; with more tiles than that the
    // (tile, trial) units are shared out evenly and a tile cut between two
    // workgroups meets in the COR running-sum buffer, which a batch leaves
    // stale (the rebuild of the window's sums rewrites it): its first P
    // doubles take the pair sums, the words after them one counter per tile
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t P = (size_t)s.N * (s.N - 1) / 2;
    const size_t words = P + ((size_t)n + 1) / 2;
    int G = n;
    double *scratch = nullptr;
    int *count = nullptr;
    if (ncu > 0 && n > ncu && s.rsum && (size_t)s.ntiles * TILE_PAIRS >= words) {
        G = ncu;
        scratch = s.rsum;
        count = (int *)(s.rsum + P);
        hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, st, (unsigned long long *)s.rsum, words);
    }
    const dim3 grid(G), blk(NT);
    switch (prec) {
    case FCX_GRAM_BF16_ID: {   // the window in BF16 once, then half the bytes per tile
        if (!s.zbf) return hipErrorInvalidValue;
        const long long n4 = (long long)K * s.N * s.Mz / 4;
        hipLaunchKernelGGL(k_z_bf16, dim3(2048), dim3(256), 0, st, s.zring, (__bf16 *)s.zbf, n4);
        hipLaunchKernelGGL((k_cor_batch<FCX_GRAM_BF16_ID, WR, WC, FCX_COR_PF16>), grid, blk, 0, st, s, K, G, scratch,
                           count);
        break;
    }
    case FCX_GRAM_BF16X3_ID:
        hipLaunchKernelGGL((k_cor_batch<FCX_GRAM_BF16X3_ID, WR, WC, FCX_COR_PF16>), grid, blk, 0, st, s, K, G,
                           scratch, count);
        break;
    default:
        hipLaunchKernelGGL((k_cor_batch<FCX_GRAM_FP32_ID, WR, WC, FCX_COR_PF32>), grid, blk, 0, st, s, K, G, scratch,
                           count);
        break;
    }
    return hipGetLastError();
}

}  // namespace fcx
