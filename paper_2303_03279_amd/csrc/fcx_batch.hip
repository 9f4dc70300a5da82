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
//   k_cor_batch     per 64x64 tile: sum over trials of the per-trial Pearson r
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
__device__ __forceinline__ __bf16 bf_hi(float x) { return (__bf16)x; }
__device__ __forceinline__ __bf16 bf_lo(float x) { return (__bf16)(x - (float)(__bf16)x); }

// One chunk of BT_CC columns of the complex Gram for a 16x16 block:
// re += Re_a Re_b + Im_a Im_b, im += Im_a Re_b - Re_a Im_b.
// X: LDS [64 nodes][BT_LD] float2; arow / bcol: this lane's A row node and
// B column node; lg = lane >> 4.
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

template <> struct Gram<FCX_GRAM_BF16_ID> {
    __device__ static void chunk(const float2 *X, int arow, int bcol, int lg, floatx4 &re, floatx4 &im)
    {
        bf16x8 ar, ai, an, br, bi;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float2 a = X[arow * BT_LD + 8 * lg + e];
            const float2 b = X[bcol * BT_LD + 8 * lg + e];
            ar[e] = (__bf16)a.x;
            ai[e] = (__bf16)a.y;
            an[e] = (__bf16)(-a.x);
            br[e] = (__bf16)b.x;
            bi[e] = (__bf16)b.y;
        }
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, bi, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(an, bi, im, 0, 0, 0);
    }
};

template <> struct Gram<FCX_GRAM_BF16X3_ID> {
    __device__ static void chunk(const float2 *X, int arow, int bcol, int lg, floatx4 &re, floatx4 &im)
    {
        bf16x8 arh, arl, aih, ail, anh, anl, brh, brl, bih, bil;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float2 a = X[arow * BT_LD + 8 * lg + e];
            const float2 b = X[bcol * BT_LD + 8 * lg + e];
            arh[e] = bf_hi(a.x);
            arl[e] = bf_lo(a.x);
            aih[e] = bf_hi(a.y);
            ail[e] = bf_lo(a.y);
            anh[e] = bf_hi(-a.x);
            anl[e] = bf_lo(-a.x);
            brh[e] = bf_hi(b.x);
            brl[e] = bf_lo(b.x);
            bih[e] = bf_hi(b.y);
            bil[e] = bf_lo(b.y);
        }
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

// ---------------------------------------------------------------- pairs
template <int PREC, int LT>
__global__ __launch_bounds__(BT_THREADS)
__attribute__((amdgpu_waves_per_eu(PREC == FCX_GRAM_FP32_ID && LT == 1 ? 4 : 1))) void k_pair_batch(SessDev<float> s,
                                                                                                     int K)
{
    __shared__ float2 Xs[64 * BT_LD];
    __shared__ float2 Us[64 * BT_LD];
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
    const bool mfmaU = needU && L == 1;
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
        floatx4 sre = {0.f, 0.f, 0.f, 0.f}, sim = sre, ure = sre, uim = sre;
        int G[4] = {0, 0, 0, 0};
        double A[4] = {0, 0, 0, 0}, Q[4] = {0, 0, 0, 0}, VUr[4] = {0, 0, 0, 0}, VUi[4] = {0, 0, 0, 0};
        for (int t0 = 0; t0 < K; t0 += TPC) {
            const int nk = min(TPC, K - t0);
            __syncthreads();
            // consecutive lanes take consecutive nodes of one column, so a
            // wavefront reads two contiguous runs of 32 nodes
            for (int e = threadIdx.x; e < 64 * BT_CC; e += BT_THREADS) {
                const int node = e & 63, col = e >> 6;
                const int t = col / L, l = col % L;
                const int g = node < 32 ? R0 + node : C0 + node - 32;
                float2 v = make_float2(0.f, 0.f), u = make_float2(0.f, 0.f);
                if (col < CC && t < nk && g < N) {
                    v = ring[(((size_t)(t0 + t) * B + b) * L + l) * N + g];
                    if (L > 1) {
                        const float wl = (float)sqrt(s.lamw[l]);
                        v.x *= wl;
                        v.y *= wl;
                    }
                    if (mfmaU) {
                        const double m2 = (double)v.x * v.x + (double)v.y * v.y;
                        const double r = m2 > 0.0 ? rsqrt(m2) : 0.0;
                        u.x = (float)(v.x * r);
                        u.y = (float)(v.y * r);
                    }
                }
                Xs[node * BT_LD + col] = v;
                if (mfmaU) Us[node * BT_LD + col] = u;
            }
            __syncthreads();
            // per-trial sums of this lane's four pairs (FP32, no contraction)
            float Ap[4] = {0.f, 0.f, 0.f, 0.f}, Qp[4] = {0.f, 0.f, 0.f, 0.f};
            if constexpr (PREC == FCX_GRAM_FP32_ID && LT == 1) {
                // FP32 Gram, one taper: each MFMA step (4 trials) is followed by
                // the vector sums of the same 4 trials, so the matrix-core
                // latency overlaps vector work.  Im(x_i conj x_j) and the Im^2
                // sum use fused multiply-adds (the kernel is bound by these
                // vector sums)
#pragma unroll
                for (int st = 0; st < BT_CC / 4; ++st) {
                    {
                        const float2 a = Xs[arow * BT_LD + 4 * st + lg];
                        const float2 bb = Xs[bcol * BT_LD + 4 * st + lg];
                        sre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, sre, 0, 0, 0);
                        sre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, sre, 0, 0, 0);
                        sim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, sim, 0, 0, 0);
                        sim = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, bb.y, sim, 0, 0, 0);
                    }
                    if (mfmaU) {
                        const float2 a = Us[arow * BT_LD + 4 * st + lg];
                        const float2 bb = Us[bcol * BT_LD + 4 * st + lg];
                        ure = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, ure, 0, 0, 0);
                        ure = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, ure, 0, 0, 0);
                        uim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, uim, 0, 0, 0);
                        uim = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, bb.y, uim, 0, 0, 0);
                    }
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        const int t = 4 * st + tt;
                        if (t < nk) {
                            const float2 xj = Xs[bcol * BT_LD + t];
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const float2 xi = Xs[rows[k] * BT_LD + t];
                                const float ci = __builtin_fmaf(xi.y, xj.x, -(xi.x * xj.y));
                                G[k] += (ci > 0.f) - (ci < 0.f);
                                Ap[k] += fabsf(ci);
                                Qp[k] = __builtin_fmaf(ci, ci, Qp[k]);
                            }
                        }
                    }
                }
            } else {
            Gram<PREC>::chunk(Xs, arow, bcol, lg, sre, sim);
            if (mfmaU) Gram<PREC>::chunk(Us, arow, bcol, lg, ure, uim);
#pragma unroll 4
            for (int t = 0; t < nk; ++t) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    float cr = 0.f, ci = 0.f;
                    for (int l = 0; l < L; ++l) {
                        const float2 xi = Xs[rows[k] * BT_LD + t * L + l];
                        const float2 xj = Xs[bcol * BT_LD + t * L + l];
                        cr = cr + (xi.x * xj.x + xi.y * xj.y);
                        ci = ci + (xi.y * xj.x - xi.x * xj.y);
                    }
                    G[k] += (ci > 0.f) - (ci < 0.f);
                    Ap[k] += fabsf(ci);
                    Qp[k] += ci * ci;
                    if (needU && L > 1) {
                        const double m2 = (double)cr * cr + (double)ci * ci;
                        if (m2 > 0.0) {
                            const double rm = rsqrt(m2);
                            VUr[k] += cr * rm;
                            VUi[k] += ci * rm;
                        }
                    }
                }
            }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                A[k] += Ap[k];
                Q[k] += Qp[k];
            }
        }
        // metrics of this bin for the lane's pairs, into the band means
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = R0 + rows[k];
            if (!(i < j && j < N)) continue;
            const double Sr = sre[k], Si = sim[k];
            const double pp = s.psd[(size_t)b * N + i] * s.psd[(size_t)b * N + j];
            if (mm & M_COH) acc[k][0] += pp > 0.0 ? (float)sqrt((Sr * Sr + Si * Si) / pp) : 0.f;
            if (mm & M_IMCOH) acc[k][1] += pp > 0.0 ? (float)(Si / sqrt(pp)) : 0.f;
            if (mm & M_PLV) {
                const double ur = mfmaU ? (double)ure[k] : VUr[k];
                const double ui = mfmaU ? (double)uim[k] : VUi[k];
                acc[k][2] += (float)(sqrt(ur * ur + ui * ui) / Kd);
            }
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
// One 64x64 tile per workgroup, 4 wavefronts each with a 32x32 quadrant
// (2x2 blocks of 16x16).  For every trial the z-scored samples of the tile's
// 64 row and 64 column nodes are staged through LDS 32 samples at a time;
// each trial's r is accumulated in FP32 by the MFMAs and added to an FP64
// sum, so the window sum carries no FP32 growth across trials.
constexpr int CR_CH = 32;
constexpr int CR_LD = CR_CH + 1;

template <int PREC>
__device__ __forceinline__ void cor_chunk(const float *Zr, const float *Zc, int ra, int cb, int lg, floatx4 &acc)
{
    if (PREC == FCX_GRAM_FP32_ID) {
#pragma unroll
        for (int st = 0; st < CR_CH / 4; ++st)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Zr[ra * CR_LD + 4 * st + lg], Zc[cb * CR_LD + 4 * st + lg], acc,
                                                       0, 0, 0);
    } else {
        bf16x8 ah, al, bh, bl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float a = Zr[ra * CR_LD + 8 * lg + e], b = Zc[cb * CR_LD + 8 * lg + e];
            if (PREC == FCX_GRAM_BF16_ID) {
                ah[e] = (__bf16)a;
                bh[e] = (__bf16)b;
            } else {
                ah[e] = bf_hi(a);
                al[e] = bf_lo(a);
                bh[e] = bf_hi(b);
                bl[e] = bf_lo(b);
            }
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
        if (PREC == FCX_GRAM_BF16X3_ID) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void k_cor_batch(SessDev<float> s, int K)
{
    __shared__ float Zr[64 * CR_LD];
    __shared__ float Zc[64 * CR_LD];
    if (s.ctl->bad) return;
    const int tile = blockIdx.x;
    const int2 tt = s.tiles[tile];
    const int I0 = tt.x * TILE, J0 = tt.y * TILE;
    const int N = s.N, Mz = s.Mz;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int qi = w >> 1, qj = w & 1;
    double R[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int k = 0; k < 4; ++k) R[a][b][k] = 0.0;
    for (int t = 0; t < K; ++t) {
        const float *z = s.zring + (size_t)t * N * Mz;
        floatx4 r[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) r[a][b] = (floatx4){0.f, 0.f, 0.f, 0.f};
        for (int n0 = 0; n0 < Mz; n0 += CR_CH) {
            __syncthreads();
            // 128 nodes x 32 samples: 8 float4 per node row chunk
            for (int e = threadIdx.x; e < 128 * (CR_CH / 4); e += 256) {
                const int node = e / (CR_CH / 4), q4 = e % (CR_CH / 4);
                const int g = node < 64 ? I0 + node : J0 + node - 64;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (g < N) v = *(const float4 *)(z + (size_t)g * Mz + n0 + 4 * q4);
                float *dst = node < 64 ? Zr + node * CR_LD : Zc + (node - 64) * CR_LD;
                dst[4 * q4 + 0] = v.x;
                dst[4 * q4 + 1] = v.y;
                dst[4 * q4 + 2] = v.z;
                dst[4 * q4 + 3] = v.w;
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    cor_chunk<PREC>(Zr, Zc, 32 * qi + 16 * a + lr, 32 * qj + 16 * b + lr, lg, r[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int k = 0; k < 4; ++k) R[a][b][k] += (double)r[a][b][k];
    }
    const size_t P = (size_t)N * (N - 1) / 2;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = I0 + 32 * qi + 16 * a + 4 * lg + k, j = J0 + 32 * qj + 16 * b + lr;
                if (!(i < j && j < N)) continue;
                const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
                s.out[7 * P + idx] = (float)(R[a][b][k] / (double)K);
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

template <int LT> static void launch_pair_batch_l(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    const dim3 grid(s.ntiles * 4), blk(BT_THREADS);
    switch (prec) {
    case FCX_GRAM_BF16_ID: hipLaunchKernelGGL((k_pair_batch<FCX_GRAM_BF16_ID, LT>), grid, blk, 0, st, s, K); break;
    case FCX_GRAM_BF16X3_ID: hipLaunchKernelGGL((k_pair_batch<FCX_GRAM_BF16X3_ID, LT>), grid, blk, 0, st, s, K); break;
    default: hipLaunchKernelGGL((k_pair_batch<FCX_GRAM_FP32_ID, LT>), grid, blk, 0, st, s, K); break;
    }
}

hipError_t launch_pair_batch(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    if (s.L == 1)
        launch_pair_batch_l<1>(s, K, prec, st);
    else
        launch_pair_batch_l<0>(s, K, prec, st);
    return hipGetLastError();
}

hipError_t launch_cor_batch(const SessDev<float> &s, int K, int prec, hipStream_t st)
{
    const dim3 grid(s.ntiles);
    switch (prec) {
    case FCX_GRAM_BF16_ID: hipLaunchKernelGGL(k_cor_batch<FCX_GRAM_BF16_ID>, grid, dim3(256), 0, st, s, K); break;
    case FCX_GRAM_BF16X3_ID: hipLaunchKernelGGL(k_cor_batch<FCX_GRAM_BF16X3_ID>, grid, dim3(256), 0, st, s, K); break;
    default: hipLaunchKernelGGL(k_cor_batch<FCX_GRAM_FP32_ID>, grid, dim3(256), 0, st, s, K); break;
    }
    return hipGetLastError();
}

}  // namespace fcx
