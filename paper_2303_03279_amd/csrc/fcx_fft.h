// Workgroup FFT in LDS and the host twiddle table, shared by the stream
// front end and the analytic-signal kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#pragma clang fp contract(off)

namespace fcx {

__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place unscaled inverse DFT (exp(+2 pi i k n / F)) of Z[F] in LDS by a
// workgroup of ST threads: radix-4 Stockham stages, one radix-2 stage when
// log2 F is odd.  Every thread of the workgroup calls it; it ends with a
// barrier.
template <int F, int ST>
__device__ void ifft_wg(float2 *Z, const float2 *__restrict__ tw)
{
    const int tid = threadIdx.x;
    constexpr int NB4 = F / 4;
    constexpr int PER4 = (NB4 + ST - 1) / ST;
    for (int Ns = 1; Ns * 4 <= F; Ns *= 4) {
        float2 v[PER4][4];
        const int step = F / (4 * Ns);
#pragma unroll
        for (int q = 0; q < PER4; ++q) {
            const int j = tid + q * ST;
            if (j < NB4) {
                const int k = j & (Ns - 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float2 a = Z[j + r * NB4];
                    if (r && Ns > 1) {
                        float2 w = tw[r * k * step];
                        w.y = -w.y;
                        a = cmulf(a, w);
                    }
                    v[q][r] = a;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER4; ++q) {
            const int j = tid + q * ST;
            if (j < NB4) {
                const int k = j & (Ns - 1);
                const float2 a0 = v[q][0], a1 = v[q][1], a2 = v[q][2], a3 = v[q][3];
                const float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
                const float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
                const float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
                const float2 d = make_float2(a1.x - a3.x, a1.y - a3.y);
                const float2 t3 = make_float2(-d.y, d.x);
                const int o = (j / Ns) * Ns * 4 + k;
                Z[o] = make_float2(t0.x + t2.x, t0.y + t2.y);
                Z[o + Ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
                Z[o + 2 * Ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
                Z[o + 3 * Ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
            }
        }
        __syncthreads();
    }
    if constexpr ((F & 0x55555555) == 0) {
        constexpr int NB2 = F / 2;
        constexpr int PER2 = (NB2 + ST - 1) / ST;
        float2 v0[PER2], v1[PER2];
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int j = tid + q * ST;
            if (j < NB2) {
                float2 w = tw[j];
                w.y = -w.y;
                v0[q] = Z[j];
                v1[q] = cmulf(Z[j + NB2], w);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int j = tid + q * ST;
            if (j < NB2) {
                Z[j] = make_float2(v0[q].x + v1[q].x, v0[q].y + v1[q].y);
                Z[j + NB2] = make_float2(v0[q].x - v1[q].x, v0[q].y - v1[q].y);
            }
        }
        __syncthreads();
    }
}

// exp(-2 pi i m / F) with the angle reduced to the first octant (host)
inline void root_of_unity(long long m, long long F, double *c, double *sn)
{
    m %= F;
    const long long q = (4 * m) / F, r = 4 * m - q * F;   // m/F = (q + r/F) / 4
    const double a = 2.0 * M_PI * (double)r / (4.0 * (double)F);
    double cc = cos(a), ss = sin(a);
    double cr, sr;
    switch (q) {
    case 0: cr = cc; sr = ss; break;
    case 1: cr = -ss; sr = cc; break;
    case 2: cr = -cc; sr = -ss; break;
    default: cr = ss; sr = -cc; break;
    }
    *c = cr;
    *sn = -sr;
}

}  // namespace fcx
