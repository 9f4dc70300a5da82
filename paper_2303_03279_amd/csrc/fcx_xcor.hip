// XCOR, the cross-correlation metric of the time-domain section, computed the
// way the implementation section describes it: spectra of the signals,
// their product, back to the time domain, then the largest correlation over
// the lags.  Per push, for the trial at the push's ring slot:
//
//   k_xcor_node   per node pair (2p, 2p + 1), from the z-scored samples z
//                 (already in the COR sample ring): the suffix energies
//                 S(tau) = sum_{t >= tau} z(t)^2 in FP64, E = S(0), the lag
//                 factors rho(tau) = sqrt(E / S(tau)), and the spectra of the
//                 unit-energy samples u = z / sqrt(E) from one FP64 FFT of
//                 length F (a power of two >= M + L) of u_2p + i u_2p+1:
//                 each node's U(f) / F for f = 0..F/2 (row operand) and the
//                 pair's D(f) = U_2p(f) - i U_2p+1(f) over the full circle
//                 (column operand), each rounded to FP32 once; the node's
//                 tail lags (below) and 1 / sqrt(S(tau))
//   k_xcor_tail   per pair: the largest XCOR over the tail lags of both
//                 nodes, summed directly in FP64.  A tail lag has
//                 S(tau) < E / 1024: there the lag factor (> 32) would
//                 magnify the FFT's rounding error beyond 1e-5, so the
//                 transform's value is not used (its lag factor is NaN)
//   k_xcor_pair   per pair-tile row i and column pair (j, j + 1): one
//                 inverse FFT of A(f) conj(D(f)), A(f) = U_i(f) / F, gives
//                 c_ij(tau) + i c_i,j+1(tau), the circular correlations of the
//                 unit-energy samples, equal to the linear ones at lags -L..L
//                 since F >= M + L; then
//                   XCOR(tau)  = c(tau) rho_i(tau)        tau = 0..L
//                   XCOR(-tau) = c(F - tau) rho_j(tau)    tau = 1..L
//                 which is c / sqrt(S_i(tau) E_j), resp. c / sqrt(E_i S_j(tau)),
//                 of the z-scored samples (0 where an energy is 0); the maximum
//                 over the 2L + 1 lags (with the tail lags' maximum), and the
//                 window sum: + this trial's
//                 maximum, - the evicted trial's maximum kept in a ring of
//                 per-trial values, so add and remove cancel exactly.
//
// The inverse FFT is a mixed-radix Stockham (autosorting) transform done by
// one wavefront in its own LDS buffer, radix 16, 16 and 4 at F = 1024 with
// the butterflies in registers.  Its first pass takes its inputs straight
// from the operands (A in LDS, D in registers, loaded while the previous
// transform ran), and its last pass hands its outputs to the maximum in
// registers, so a transform makes two trips through LDS.  The lag factors
// carry NaN at the output indices that are no lag, which the maximum skips.
#include "fcx_device.h"

#include <math.h>

#pragma clang fp contract(off)

namespace fcx {

constexpr int XT = 256;   // threads of the node kernel

// ---------------------------------------------------------------------------
// node pass: one workgroup per node pair
// ---------------------------------------------------------------------------
template <typename T, int F>
__global__ __launch_bounds__(XT) void k_xcor_node(SessDev<T> s)
{
    __shared__ double2 buf[2][F];
    __shared__ float z[2][F];
    if (s.ctl->bad) return;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int N = s.N, M = s.M, L = s.xL;
    const int n0 = 2 * p;
    const bool has1 = n0 + 1 < N;
    const PushView pv = push_view(s, s.ctl->pushed);
    const float *zr = s.zring + ((size_t)pv.slot_new * N + n0) * s.Mz;
    // per node: the first tail lag (M: none) and 1 + the last nonzero sample
    __shared__ int tail_lo[2], tail_end[2];
    if (tid < 2) {
        tail_lo[tid] = M;
        tail_end[tid] = 0;
    }
    for (int t = tid; t < M; t += XT) {
        z[0][t] = zr[t];
        z[1][t] = has1 ? zr[s.Mz + t] : 0.f;
    }
    __syncthreads();
    {
        int e0 = 0, e1 = 0;
        for (int t = tid; t < M; t += XT) {
            if (z[0][t] != 0.f) e0 = t + 1;
            if (z[1][t] != 0.f) e1 = t + 1;
        }
        for (int o = 32; o > 0; o >>= 1) {
            e0 = max(e0, __shfl_xor(e0, o, 64));
            e1 = max(e1, __shfl_xor(e1, o, 64));
        }
        if (lane == 0) {
            if (e0) atomicMax(&tail_end[0], e0);
            if (e1) atomicMax(&tail_end[1], e1);
        }
    }
    // suffix energies, FP64, wavefront h for node h: lane l sums its segment
    // of samples from the top, the sum of the segments above it comes from a
    // scan over the lanes (fixed order), then the lane writes its segment's
    // suffix sums
    double *suf = reinterpret_cast<double *>(buf[1]);   // [2][F]
    if (wv < 2) {
        const int h = wv;
        const int seg = (M + 63) / 64;
        const int t0 = lane * seg, t1 = min(M, t0 + seg);
        double part = 0.0;
        for (int t = t1 - 1; t >= t0; --t) part += (double)z[h][t] * (double)z[h][t];
        double above = __shfl_down(part, 1, 64);
        if (lane == 63) above = 0.0;
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_down(above, off, 64);
            if (lane + off < 64) above += o;
        }
        double acc = above;
        for (int t = t1 - 1; t >= t0; --t) {
            acc += (double)z[h][t] * (double)z[h][t];
            suf[h * F + t] = acc;
        }
    }
    __syncthreads();
    const double E0 = suf[0], E1 = suf[F];
    // tail lags: 1 <= tau <= L with 0 < S(tau) < E / XCOR_TAIL_RHO2; S does
    // not increase with tau, so they run from the first such lag to the
    // last lag with S > 0 (tau < tail_end)
    {
        int a0 = M, a1 = M;
        for (int tau = 1 + tid; tau <= min(L, M - 1); tau += XT) {
            if (tau < a0 && tau < tail_end[0] && suf[tau] * XCOR_TAIL_RHO2 < suf[0]) a0 = tau;
            if (tau < a1 && tau < tail_end[1] && suf[F + tau] * XCOR_TAIL_RHO2 < suf[F]) a1 = tau;
        }
        for (int o = 32; o > 0; o >>= 1) {
            a0 = min(a0, __shfl_xor(a0, o, 64));
            a1 = min(a1, __shfl_xor(a1, o, 64));
        }
        if (lane == 0) {
            if (a0 < M) atomicMin(&tail_lo[0], a0);
            if (a1 < M) atomicMin(&tail_lo[1], a1);
        }
    }
    __syncthreads();
    if (tid < 2) {
        const int a = tail_lo[tid], e = tail_end[tid];
        s.xtail[n0 + tid] = a < min(e, L + 1) ? make_int2(a, e) : make_int2(0, 0);
    }
    for (int e = tid; e < 2 * s.Mz; e += XT) {
        const int h = e >= s.Mz, t = e - h * s.Mz;
        const double S = t < M ? suf[h * F + t] : 0.0;
        s.xg[(size_t)(n0 + h) * s.Mz + t] = S > 0.0 ? 1.0 / sqrt(S) : 0.0;
    }
    // lag factors: index tau < F/2 for lag tau, index F - tau for lag -tau
    for (int e = tid; e < 2 * F; e += XT) {
        const int h = e / F, id = e - h * F;
        const int tau = id < F / 2 ? id : F - id;
        float v = __builtin_nanf("");
        if (tau <= L && !(tau >= tail_lo[h] && tau < tail_end[h])) {
            const double S = suf[h * F + tau];
            v = S > 0.0 ? (float)sqrt(suf[h * F] / S) : 0.f;
        }
        s.xrho[(size_t)(n0 + h) * F + id] = v;
    }
    const double r0 = E0 > 0.0 ? 1.0 / sqrt(E0) : 0.0, r1 = E1 > 0.0 ? 1.0 / sqrt(E1) : 0.0;
    for (int t = tid; t < F; t += XT)
        buf[0][t] = t < M ? make_double2(r0 * (double)z[0][t], r1 * (double)z[1][t]) : make_double2(0.0, 0.0);
    __syncthreads();
    // forward FFT, radix-2 Stockham passes between the two buffers
    int src = 0;
    for (int ns = 1; ns < F; ns *= 2) {
        const double2 *in = buf[src];
        double2 *out = buf[src ^ 1];
        for (int j = tid; j < F / 2; j += XT) {
            const int k = j & (ns - 1);
            const double2 a0 = in[j], b = in[j + F / 2];
            const double2 w = s.xtw[k * (F / (2 * ns))];   // exp(-2 pi i k / (2 ns))
            const double2 a1 = make_double2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
            const int o = 2 * (j - k) + k;                  // (j / ns) 2 ns + k
            out[o] = make_double2(a0.x + a1.x, a0.y + a1.y);
            out[o + ns] = make_double2(a0.x - a1.x, a0.y - a1.y);
        }
        __syncthreads();
        src ^= 1;
    }
    // Y = U0 + i U1: D(f) = U0(f) - i U1(f) = conj(Y(F - f)),
    // U0(f) = (Y(f) + conj(Y(F - f))) / 2, U1(f) = (Y(f) - conj(Y(F - f))) / 2i
    const double2 *Y = buf[src];
    const double sc = 0.5 / (double)F;
    float2 *x0 = s.xspec + (size_t)n0 * (F / 2 + 1), *x1 = x0 + (F / 2 + 1);
    for (int f = tid; f < F; f += XT) {
        const double2 y = Y[f], ym = Y[(F - f) & (F - 1)];
        s.xpair[(size_t)p * F + f] = make_float2((float)ym.x, (float)-ym.y);
        if (f <= F / 2) {
            x0[f] = make_float2((float)((y.x + ym.x) * sc), (float)((y.y - ym.y) * sc));
            x1[f] = make_float2((float)((y.y + ym.y) * sc), (float)((ym.x - y.x) * sc));
        }
    }
}

// ---------------------------------------------------------------------------
// tail lags: one lane per column, four rows of a tile per wavefront
// ---------------------------------------------------------------------------
// The largest XCOR over the tail lags of the pair (i, j): lags tau of row
// node i's tail, sum_t z_i(t + tau) z_j(t) / sqrt(S_i(tau) E_j), and lags
// -tau of column node j's tail, sum_t z_i(t) z_j(t + tau) / sqrt(E_i S_j(tau)),
// summed in FP64 from the trial's z-scored samples (products of FP32 values
// are exact in FP64).  The sums stop at the node's last nonzero sample.  A
// wavefront takes four rows, so one column's samples serve four pairs.
constexpr int XTAIL_RPW = 4;                      // rows per wavefront
constexpr int XTAIL_WAVES = 4;                    // wavefronts per workgroup
constexpr int XTAIL_ROWS = XTAIL_RPW * XTAIL_WAVES;   // rows per workgroup

template <typename T>
__global__ __launch_bounds__(64 * XTAIL_WAVES) void k_xcor_tail(SessDev<T> s)
{
    if (s.ctl->bad) return;
    const int tile = blockIdx.x / (TILE / XTAIL_ROWS);
    const int r0 = (blockIdx.x % (TILE / XTAIL_ROWS)) * XTAIL_ROWS +
                   XTAIL_RPW * (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int2 tt = s.tiles[tile];
    const int N = s.N, L = s.xL, Mz = s.Mz;
    const int i0 = tt.x * TILE + r0, j = tt.y * TILE + lane;
    float best[XTAIL_RPW];
#pragma unroll
    for (int k = 0; k < XTAIL_RPW; ++k) best[k] = __builtin_nanf("");
    if (i0 < N && j > i0 && j < N) {
        const PushView pv = push_view(s, s.ctl->pushed);
        const float *zs = s.zring + (size_t)pv.slot_new * N * Mz;
        const float *zj = zs + (size_t)j * Mz;
        const double *gj = s.xg + (size_t)j * Mz;
        const double gj0 = gj[0];
        const int2 tj = s.xtail[j];
        const int nr = min(XTAIL_RPW, N - i0);   // rows of this wavefront below N
        // lags tau >= 0 in each row's tail
#pragma unroll
        for (int k = 0; k < XTAIL_RPW; ++k) {
            if (k >= nr) break;
            const int i = i0 + k;
            if (j <= i) continue;
            const float *zi = zs + (size_t)i * Mz;
            const double *gi = s.xg + (size_t)i * Mz;
            const int2 ti = s.xtail[i];
            for (int tau = ti.x; tau < min(ti.y, L + 1); ++tau) {
                double acc = 0.0;
                for (int t = 0; t < ti.y - tau; ++t) acc = __builtin_fma((double)zi[t + tau], (double)zj[t], acc);
                best[k] = fmaxf(best[k], (float)(acc * gi[tau] * gj0));
            }
        }
        // lags -tau in the column's tail, for the four rows at once
        for (int tau = tj.x; tau < min(tj.y, L + 1); ++tau) {
            double acc[XTAIL_RPW];
#pragma unroll
            for (int k = 0; k < XTAIL_RPW; ++k) acc[k] = 0.0;
            for (int t = 0; t < tj.y - tau; ++t) {
                const double v = (double)zj[t + tau];
#pragma unroll
                for (int k = 0; k < XTAIL_RPW; ++k)
                    if (k < nr) acc[k] = __builtin_fma((double)zs[(size_t)(i0 + k) * Mz + t], v, acc[k]);
            }
            const double g = gj[tau];
#pragma unroll
            for (int k = 0; k < XTAIL_RPW; ++k)
                if (k < nr && j > i0 + k)
                    best[k] = fmaxf(best[k], (float)(acc[k] * g * s.xg[(size_t)(i0 + k) * Mz]));
        }
    }
#pragma unroll
    for (int k = 0; k < XTAIL_RPW; ++k)
        s.xtm[(size_t)tile * TILE_PAIRS + (size_t)(r0 + k) * TILE + lane] = best[k];
}

// ---------------------------------------------------------------------------
// pair pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// a conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.y, b.x, -(a.x * b.y)));
}

// A transform buffer holds element m at m + m / 16: the pad after every 16
// elements (128 bytes) spreads the strided loads and stores over the LDS
// banks (measured: fewer conflicts than a pad every 8, 32 or 64 elements).
constexpr int XPAD_SHIFT = 4;
__host__ __device__ constexpr int xpad(int m) { return m + (m >> XPAD_SHIFT); }
template <int F> constexpr int xbuf_len() { return F + (F >> XPAD_SHIFT); }

// exp(+2 pi i m / 16), m = 0..7
__constant__ const float W16_RE[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__constant__ const float W16_IM[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                      1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// o exp(+2 pi i m / R), m < R / 2 known at compile time after unrolling:
// no arithmetic for m = 0 and for the quarter turn
template <int R>
__device__ __forceinline__ float2 wrot(float2 o, int m)
{
    if (m == 0) return o;
    if (4 * m == R) return make_float2(-o.y, o.x);
    const int w = m * (16 / R);
    return cmul(o, make_float2(W16_RE[w], W16_IM[w]));
}

// In-register inverse DFT of R = 4, 8 or 16 points: y_m = sum_r v_r
// exp(+2 pi i r m / R), split into even and odd halves down to radix 4.
template <int R>
__device__ __forceinline__ void idft_reg(float2 (&v)[R])
{
    if constexpr (R == 4) {
        const float2 t0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 t1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 t2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        const float2 t3 = make_float2(-d.y, d.x);    // +i (v1 - v3)
        v[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        v[1] = make_float2(t1.x + t3.x, t1.y + t3.y);
        v[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        v[3] = make_float2(t1.x - t3.x, t1.y - t3.y);
    } else {
        constexpr int H = R / 2;
        float2 e[H], o[H];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            e[m] = v[2 * m];
            o[m] = v[2 * m + 1];
        }
        idft_reg<H>(e);
        idft_reg<H>(o);
        constexpr float C = 0.70710678118654752f;   // sqrt(1/2)
#pragma unroll
        for (int m = 0; m < H; ++m) {
            if (8 * m == R || 8 * m == 3 * R) {
                // exp(+2 pi i m / R) = (+-C, C): e +- o w from o.x - o.y and
                // o.x + o.y by fused multiply-adds
                const float dx = o[m].x - o[m].y, sx = o[m].x + o[m].y;
                if (8 * m == R) {   // w = (C, C): o w = (C dx, C sx)
                    v[m] = make_float2(__builtin_fmaf(C, dx, e[m].x), __builtin_fmaf(C, sx, e[m].y));
                    v[m + H] = make_float2(__builtin_fmaf(-C, dx, e[m].x), __builtin_fmaf(-C, sx, e[m].y));
                } else {            // w = (-C, C): o w = (-C sx, C dx)
                    v[m] = make_float2(__builtin_fmaf(-C, sx, e[m].x), __builtin_fmaf(C, dx, e[m].y));
                    v[m + H] = make_float2(__builtin_fmaf(C, sx, e[m].x), __builtin_fmaf(-C, dx, e[m].y));
                }
            } else {
                const float2 t = wrot<R>(o[m], m);
                v[m] = make_float2(e[m].x + t.x, e[m].y + t.y);
                v[m + H] = make_float2(e[m].x - t.x, e[m].y - t.y);
            }
        }
    }
}

// Stockham pass of radix R over stride NS (product of the radices before it):
// butterfly j takes Z[j + r F / R] (times exp(+2 pi i r k / (R NS)),
// k = j mod NS, from the table T laid out [r - 1][k]) and its R-point DFT
// goes to Z[(j / NS) NS R + k + m NS].  Loads: xpass_load; the DFT and the
// stores: xpass_store.  A wavefront's LDS operations are performed in order,
// so all loads of a pass precede its stores; the wave barriers keep the
// compiler from moving LDS accesses across the phase boundaries.  With the
// pad every 16 elements both address patterns are one base plus constants
// (F / R and NS are multiples of 16, or NS < 16 with k + (m NS mod 16) < 16).
template <int F, int R, int NS>
__device__ __forceinline__ void xpass_load(const float2 *Z, const float2 *T, int lane,
                                           float2 (&v)[F / R / 64][R])
{
    constexpr int NB = F / R, PER = NB / 64;
    static_assert(NB % 64 == 0 && NB % 32 == 0, "butterflies per lane");
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + 64 * q;
        const int k = j & (NS - 1);
        const float2 *zi = Z + xpad(j);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float2 a = zi[r * NB + ((r * NB) >> XPAD_SHIFT)];
            if (NS > 1 && r) a = cmul(a, T[(r - 1) * NS + k]);
            v[q][r] = a;
        }
    }
}

template <int F, int R, int NS>
__device__ __forceinline__ void xpass_store(float2 *Z, int lane, float2 (&v)[F / R / 64][R])
{
    constexpr int PER = F / R / 64;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + 64 * q;
        const int k = j & (NS - 1);
        idft_reg<R>(v[q]);
        float2 *zo = Z + xpad((j / NS) * NS * R + k);
#pragma unroll
        for (int m = 0; m < R; ++m) zo[m * NS + ((m * NS) >> XPAD_SHIFT)] = v[q][m];
    }
}

template <int F, int R, int NS>
__device__ __forceinline__ void xpass(float2 *Z, const float2 *T, int lane)
{
    float2 v[F / R / 64][R];
    xpass_load<F, R, NS>(Z, T, lane, v);
    __builtin_amdgcn_wave_barrier();
    xpass_store<F, R, NS>(Z, lane, v);
    __builtin_amdgcn_wave_barrier();
}

// Largest value over the wavefront (no NaN in v), the same in every lane:
// within each 16-lane row by v_max_f32 with DPP rotations of its first
// operand (8, 4, 2, 1; two wait states before each DPP read of a VGPR the
// previous instruction wrote, and before the value leaves the block), then
// the four rows' maxima read from lanes 0, 16, 32 and 48
__device__ __forceinline__ float wave_max(float v)
{
    float r;
    asm volatile(
        "s_nop 1\n"
        "v_max_f32_dpp %0, %1, %1 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "s_nop 1\n"
        "v_max_f32_dpp %0, %0, %0 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "s_nop 1\n"
        "v_max_f32_dpp %0, %0, %0 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "s_nop 1\n"
        "v_max_f32_dpp %0, %0, %0 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "s_nop 1"
        : "=&v"(r)
        : "v"(v));
    const int b = __builtin_bit_cast(int, r);
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48));
    return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// waves per workgroup of the pair kernel (each has its own transform buffer)
template <int F> constexpr int xcor_waves() { return F >= 2048 ? 2 : 4; }

// One workgroup per (tile, row of the tile): row node i against the tile's
// columns j > i, two columns (a node pair 2p, 2p + 1) per transform.  The
// row operand A (full circle), the twiddles and the row's lag factors are
// set up once; each wavefront takes column pairs in turn into its own
// transform buffer, loading the next pair's D into registers while it
// transforms the current one.
template <typename T, int F>
__global__ __launch_bounds__(64 * xcor_waves<F>()) __attribute__((amdgpu_waves_per_eu(F == 1024 ? 3 : 1)))
void k_xcor_pair(SessDev<T> s)
{
    constexpr int NW = xcor_waves<F>();
    constexpr int R1 = xcor_r1(F), NB1 = F / R1, PER1 = NB1 / 64;
    constexpr int NP = xcor_npass(F);
    constexpr int RL = xcor_pass_r(F, NP - 1), NSL = xcor_pass_ns(F, NP - 1), PERL = NSL / 64;
    constexpr int HL = RL / 2;   // outputs m < HL of the last pass are lags >= 0, the rest lags < 0
    static_assert(NSL * RL == F, "last pass");
    __shared__ float2 Zw[NW][xbuf_len<F>()];
    __shared__ float2 A[F];
    __shared__ float2 tws[xcor_tw_len(F)];
    // the row's 64 pairs of this tile: window sum, evicted trial's maximum,
    // tail lags' maximum (loaded with the row operand, read by the jobs)
    __shared__ double wsum[TILE];
    __shared__ float wold[TILE], wtm[TILE];
    if (s.ctl->bad) return;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int tile = item / TILE, r = item % TILE;
    const int2 tt = s.tiles[tile];
    const int N = s.N, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: job indices live in scalar registers
    const int i = tt.x * TILE + r, J0 = tt.y * TILE;
    if (i >= N) return;
    // column pairs (J0 + 2p, J0 + 2p + 1) that hold a column j > i, j < N
    const int jend = min(J0 + TILE, N);
    const int plo = (max(J0, i + 1) - J0) >> 1, phi = (jend - J0 + 1) >> 1;
    if (plo >= phi) return;
    const PushView pv = push_view(s, s.ctl->pushed);
    {
        const float2 *xs = s.xspec + (size_t)i * (F / 2 + 1);
        for (int f = tid; f < F; f += 64 * NW) {
            const float2 a = xs[f <= F / 2 ? f : F - f];
            A[f] = f <= F / 2 ? a : make_float2(a.x, -a.y);
        }
        for (int e = tid; e < xcor_tw_len(F); e += 64 * NW) tws[e] = s.xtwi[e];
        if (tid < TILE) {
            const int jj = J0 + tid;
            const size_t e = (size_t)tile * TILE_PAIRS + (size_t)r * TILE + tid;
            double sm = 0.0;
            float vo = 0.f, tm = 0.f;
            if (jj > i && jj < N) {
                sm = s.xsum[e];
                if (pv.has_old) vo = s.xval[(size_t)pv.slot_old * s.ntiles * TILE_PAIRS + e];
                tm = s.xtm[e];
            }
            wsum[tid] = sm;
            wold[tid] = vo;
            wtm[tid] = tm;
        }
    }
    // the column operands and lag factors through buffer resources: a uniform
    // job offset in a scalar register, the lane's offset, constants
    const int np = (N + 1) / 2;
    const Rsrc dres = tile_rsrc(s.xpair, (uint32_t)((size_t)np * F * 8));
    const Rsrc rres = tile_rsrc(s.xrho, (uint32_t)((size_t)2 * np * F * 4));
    // the row's lag factors at this lane's outputs of lags >= 0
    float rowf[PERL][HL];
#pragma unroll
    for (int q = 0; q < PERL; ++q)
#pragma unroll
        for (int m = 0; m < HL; ++m)
            rowf[q][m] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rres, 4 * (lane + 64 * q + NSL * m), i * F * 4, 0));
    __syncthreads();
    float2 *Z = Zw[wv];
    const size_t TP = (size_t)s.ntiles * TILE_PAIRS;
    const size_t P = (size_t)N * (N - 1) / 2;
    const double invK = 1.0 / (double)pv.K;
    const int c0 = (J0 >> 1);   // node pair index of column J0
    auto load_d = [&](int pp, float2 (&d)[PER1][R1]) {
#pragma unroll
        for (int q = 0; q < PER1; ++q)
#pragma unroll
            for (int rr = 0; rr < R1; ++rr)
                d[q][rr] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                                          dres, 8 * (lane + 64 * q), ((c0 + pp) * F + NB1 * rr) * 8, 0));
    };
    // one column pair: transform with operand d, loading the operand of pair
    // pn (if any) into dn once d is consumed
    auto job = [&](int pp, float2 (&d)[PER1][R1], int pn, float2 (&dn)[PER1][R1]) {
        const int j1 = J0 + 2 * pp, j2 = j1 + 1;
        // lanes 0 and 1: pairs (i, j1) and (i, j2)
        const size_t e = (size_t)tile * TILE_PAIRS + (size_t)r * TILE + (j1 + lane - J0);
        // this job's column lag factors (lags < 0), used after the transform
        float cf1[PERL][HL], cf2[PERL][HL];
#pragma unroll
        for (int q = 0; q < PERL; ++q)
#pragma unroll
            for (int m = 0; m < HL; ++m) {
                const int o = 4 * (lane + 64 * q);
                cf1[q][m] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rres, o, (j1 * F + NSL * (m + HL)) * 4, 0));
                cf2[q][m] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(rres, o, (j2 * F + NSL * (m + HL)) * 4, 0));
            }
        // first pass: inputs A(f) conj(D(f)) at f = b + NB1 r
        {
            float2 v[PER1][R1];
#pragma unroll
            for (int q = 0; q < PER1; ++q)
#pragma unroll
                for (int rr = 0; rr < R1; ++rr) v[q][rr] = cmulc(A[lane + 64 * q + NB1 * rr], d[q][rr]);
            if (pn < phi) load_d(pn, dn);
            xpass_store<F, R1, 1>(Z, lane, v);
            __builtin_amdgcn_wave_barrier();
        }
        // middle passes
        if constexpr (NP == 3) xpass<F, xcor_pass_r(F, 0), xcor_pass_ns(F, 0)>(Z, tws + xcor_tw_off(F, 0), lane);
        if constexpr (NP == 3) xpass<F, xcor_pass_r(F, 1), xcor_pass_ns(F, 1)>(Z, tws + xcor_tw_off(F, 1), lane);
        if constexpr (NP == 2) xpass<F, xcor_pass_r(F, 0), xcor_pass_ns(F, 0)>(Z, tws + xcor_tw_off(F, 0), lane);
        // last pass: its outputs j + NSL m (j = lane + 64 q) stay in registers
        float2 y[PERL][RL];
        xpass_load<F, RL, NSL>(Z, tws + xcor_tw_off(F, NP - 1), lane, y);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < PERL; ++q) idft_reg<RL>(y[q]);
        // largest XCOR over the lags of both pairs (the factors are NaN at
        // indices of no lag, which fmaxf skips)
        float b1 = -INFINITY, b2 = -INFINITY, e1 = -INFINITY, e2 = -INFINITY;
#pragma unroll
        for (int q = 0; q < PERL; ++q)
#pragma unroll
            for (int m = 0; m < RL; ++m) {
                const float f1 = m < HL ? rowf[q][m] : cf1[q][m - HL];
                const float f2 = m < HL ? rowf[q][m] : cf2[q][m - HL];
                if (m & 1) {
                    e1 = fmaxf(e1, y[q][m].x * f1);
                    e2 = fmaxf(e2, y[q][m].y * f2);
                } else {
                    b1 = fmaxf(b1, y[q][m].x * f1);
                    b2 = fmaxf(b2, y[q][m].y * f2);
                }
            }
        b1 = wave_max(fmaxf(b1, e1));
        b2 = wave_max(fmaxf(b2, e2));
        if (lane < 2) {
            const int jj = lane == 0 ? j1 : j2;
            if (jj > i && jj < N) {
                const int c = jj - J0;
                const float v = fmaxf(lane == 0 ? b1 : b2, wtm[c]);   // the tail lags (NaN: none)
                double sum = wsum[c] + (double)v;
                if (pv.has_old) sum = sum - (double)wold[c];
                s.xsum[e] = sum;
                s.xval[(size_t)pv.slot_new * TP + e] = v;
                const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(jj - i - 1);
                s.out[8 * P + idx] = (T)(sum * invK);
            }
        }
        __builtin_amdgcn_wave_barrier();   // Z is rebuilt for the next columns
    };
    // the jobs of this wavefront two at a time, the operand registers
    // alternating, so the loads of the next operand need no copies
    float2 d0[PER1][R1], d1[PER1][R1];
    int pp = plo + wv;
    if (pp < phi) load_d(pp, d0);
    for (; pp < phi; pp += 2 * NW) {
        job(pp, d0, pp + NW, d1);
        if (pp + NW >= phi) break;
        job(pp + NW, d1, pp + 2 * NW, d0);
    }
}

template <typename T, int F> static void launch_xcor_f(const SessDev<T> &s, hipStream_t st)
{
    hipLaunchKernelGGL((k_xcor_node<T, F>), dim3((s.N + 1) / 2), dim3(XT), 0, st, s);
    hipLaunchKernelGGL((k_xcor_tail<T>), dim3((unsigned)(s.ntiles * (TILE / XTAIL_ROWS))), dim3(64 * XTAIL_WAVES),
                       0, st, s);
    hipLaunchKernelGGL((k_xcor_pair<T, F>), dim3((unsigned)(s.ntiles * TILE)), dim3(64 * xcor_waves<F>()), 0, st,
                       s);
}

template <typename T> hipError_t launch_xcor(const SessDev<T> &s, hipStream_t st)
{
    // the lag ranges of the last pass's output halves: L < F / 2
    if (2 * s.xL >= s.xF) return hipErrorInvalidValue;
    switch (s.xF) {
    case 256: launch_xcor_f<T, 256>(s, st); break;
    case 512: launch_xcor_f<T, 512>(s, st); break;
    case 1024: launch_xcor_f<T, 1024>(s, st); break;
    case 2048: launch_xcor_f<T, 2048>(s, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_xcor<float>(const SessDev<float> &, hipStream_t);
template hipError_t launch_xcor<double>(const SessDev<double> &, hipStream_t);

}  // namespace fcx
