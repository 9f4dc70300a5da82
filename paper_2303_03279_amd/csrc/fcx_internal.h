// Internal declarations shared by the host session code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcx {

constexpr int TILE = 64;             // pair tile edge: a tile holds 64 x 64 pairs
constexpr int TILE_PAIRS = TILE * TILE;
constexpr int PAIR_THREADS = 256;    // workgroup of the pair kernels (4 waves)
constexpr int SLICE_ROWS = 16;       // a workgroup owns a 16-row slice of a tile
constexpr int SLICES = TILE / SLICE_ROWS;
constexpr int PAIR_NODES = SLICE_ROWS + TILE;   // row + column nodes staged per slice
constexpr int PAIR_LDS_BYTES = 40 * 1024;
constexpr int ZPAD = 32;             // COR sample rows padded to a multiple of 32

// running-sum planes of the pair state: FP64, except the unit-phasor sums of
// FP32 sessions (int32 fixed point) and the sign sums (int8 or int16)
enum Plane { P_SRE = 0, P_SIM = 1, P_URE = 2, P_UIM = 3, P_A = 4, P_Q = 5, NPLANES = 6 };

// Gram precisions (same values as the public header)
enum { FCX_GRAM_FP32_ID = 0, FCX_GRAM_BF16_ID = 1, FCX_GRAM_BF16X3_ID = 2 };

// metric bits (same values as the public header)
enum : uint32_t { M_COH = 1, M_IMCOH = 2, M_PLV = 4, M_PLI = 8, M_WPLI = 16, M_USPLI = 32,
                  M_DSWPLI = 64, M_COR = 128, M_XCOR = 256 };

// XCOR: largest FFT length (LDS of one wavefront's transform)
constexpr int XCOR_MAX_F = 2048;
// XCOR tail lags: the lags tau of a node whose suffix energy S(tau) is below
// E / XCOR_TAIL_RHO2 (lag factor sqrt(E / S(tau)) above 32).  The FP32 FFT's
// absolute error in the unit-energy correlation, about 1e-7, grows by that
// factor, so these lags are summed directly in FP64 instead.
constexpr double XCOR_TAIL_RHO2 = 1024.0;

// XCOR inverse FFT of length F (256..2048) by one wavefront: a first pass of
// radix xcor_r1(F), then xcor_npass(F) passes of radix xcor_pass_r(F, i) over
// strides xcor_pass_ns(F, i) (product of the radices before it).  The
// twiddles of those passes, exp(+2 pi i r k / (R NS)) for r = 1..R-1 and
// k < NS, are stored pass after pass, [r - 1][k] within a pass, in a table of
// xcor_tw_len(F) entries.
__host__ __device__ constexpr int xcor_r1(int F) { return F >= 1024 ? 16 : F / 64; }
__host__ __device__ constexpr int xcor_npass(int F) { return F == 256 ? 3 : 2; }
__host__ __device__ constexpr int xcor_pass_r(int F, int i)
{
    return F == 256 ? 4 : F == 512 ? 8 : i == 0 ? 16 : F / 256;
}
__host__ __device__ constexpr int xcor_pass_ns(int F, int i)
{
    return F == 256 ? (i == 0 ? 4 : i == 1 ? 16 : 64) : F == 512 ? (i == 0 ? 8 : 64) : (i == 0 ? 16 : 256);
}
__host__ __device__ constexpr int xcor_tw_off(int F, int i)
{
    return i == 0 ? 0 : xcor_tw_off(F, i - 1) + (xcor_pass_r(F, i - 1) - 1) * xcor_pass_ns(F, i - 1);
}
__host__ __device__ constexpr int xcor_tw_len(int F) { return xcor_tw_off(F, xcor_npass(F)); }

// Device-resident push control.  Every kernel of a push reads it; only the
// commit kernel advances it, so a rejected (non-finite) trial changes nothing.
struct DevCtl {
    long long pushed;     // trials accepted so far
    int bad;              // set by the spectra kernel when the trial is not finite
    int pad;
    long long rejected;   // trials rejected so far
};

// Everything a kernel needs to know about one session (passed by value, or
// from a device array of descriptors in the serving path).
template <typename T>
struct SessDev {
    int N, M, W, B, L, nT, ntiles, Mz;
    uint32_t metrics;
    int has_cor;
    const int2 *tiles;      // [ntiles] (tile row, tile col), row <= col
    T *ring;                // [(W+1)][B][L][N] complex (re, im interleaved)
    double *psd;            // [B][N] running sum of per-trial power
    void *plane[NPLANES];   // [ntiles][B][TILE_PAIRS] or null when not needed
    void *gsum;             // [ntiles][B][TILE_PAIRS] sign sums (int8 or int16) or null
    int u_fixed;            // unit-phasor planes hold int32 multiples of 2^-ufix_bits
    int ufix_bits;
    int g_narrow;           // sign sums are int8
    T *out;                 // [8][P] band-mean networks
    DevCtl *ctl;
    const T *wtw;           // [L][B][M] complex taper * exp(-2 pi i k n / F)
    const double *lamw;     // [L] taper weights, normalised to sum 1
    const void *x;          // current trial input [N][ldx] (T)
    long long ldx;
    float *zring;           // [(W+1)][N][Mz] z-scored samples (COR)
    void *zbf;              // [W][N][Mz] BF16 copy of a batch window's z-scored samples
                            // (BF16 COR batch), or null
    double *rsum;           // [ntiles][TILE_PAIRS] running sum of per-trial r (COR)
    long long kbase;        // -1: sliding push; >= 0: replay of a cached window
                            // (add only, K = pushed - kbase + 1)
    int R;                  // ring slots (>= W + 1); trial tp sits in slot tp mod R
    int nt;                 // trials one pass applies, in order (1 except for a
                            // served session's coalesced group; x then holds nt
                            // trials, N x ldx elements apart)
    int xL, xF;             // XCOR: lags -xL..xL, FFT length (power of 2 >= M + xL)
    const double2 *xtw;     // [xF] exp(-2 pi i m / xF)
    const float2 *xtwi;     // [xcor_tw_len(xF)] twiddles of the inverse FFT's passes
    // the trial's z-scored samples of node n scaled to unit energy (u = z / sqrt(E),
    // E = sum z^2; u = 0 if E = 0), for N rounded up to even (a missing last
    // node is 0):
    float2 *xspec;          // [N][xF/2+1] U(f) / xF, f = 0..xF/2
    float2 *xpair;          // [N/2][xF] U_2p(f) - i U_2p+1(f) over the full circle
    float *xrho;            // [N][xF] lag factor sqrt(E / S(tau)), S(tau) = sum_{t >= tau} z^2,
                            // at index tau (tau <= xL) and xF - tau (1 <= tau <= xL);
                            // 0 where S = 0, NaN at the indices of no lag and of tail lags
    int2 *xtail;            // [N] (a, e): the node's tail lags are a <= tau < min(e, xL + 1),
                            // e = 1 + its last nonzero sample; (0, 0): none
    double *xg;             // [N][Mz] 1 / sqrt(S(tau)) (0 where S = 0)
    float *xtm;             // [ntiles][TILE_PAIRS] largest XCOR over the tail lags of both
                            // nodes of the pair (NaN: no tail lag)
    float *xval;            // [(W+1)][ntiles][TILE_PAIRS] per-trial XCOR maxima
    double *xsum;           // [ntiles][TILE_PAIRS] their running sum over the window
};

// Which ring slots a push touches and how many trials the window holds after it.
struct PushView {
    long long tp;   // index of the trial being added
    int K;          // trials in the window after the update
    int slot_new, slot_old;
    bool has_old;   // a trial is evicted
};

template <typename T>
__host__ __device__ inline PushView push_view(const SessDev<T> &s, long long tp)
{
    PushView v;
    v.tp = tp;
    if (s.kbase >= 0) {
        v.has_old = false;
        v.K = (int)(tp - s.kbase + 1);
    } else {
        v.has_old = tp >= s.W;
        v.K = v.has_old ? s.W : (int)tp + 1;
    }
    v.slot_new = (int)(tp % (long long)s.R);
    v.slot_old = v.has_old ? (int)((tp - s.W) % (long long)s.R) : 0;
    return v;
}

// launchers (implemented in fcx_kernels.hip); all return hipError_t
template <typename T> hipError_t launch_spectra(const SessDev<T> &s, hipStream_t st);
template <typename T> hipError_t launch_psd(const SessDev<T> &s, hipStream_t st);
template <typename T> hipError_t launch_pair_update(const SessDev<T> &s, hipStream_t st);
template <typename T> hipError_t launch_znorm(const SessDev<T> &s, hipStream_t st);
// the running sums (pair planes, COR sums, networks; power sums) of the K
// cached trials first .. first + K - 1 rebuilt in one pass, bit for bit the
// sums a replay of those pushes from zero gives
template <typename T> hipError_t launch_pair_rebuild(const SessDev<T> &s, long long first, int K, hipStream_t st);
template <typename T> hipError_t launch_psd_rebuild(const SessDev<T> &s, long long first, int K, hipStream_t st);
// trials k = 0..K-1 of a device-resident batch (at x + k * stride elements)
// into ring slot k
template <typename T> hipError_t launch_spectra_batch(const SessDev<T> &s, int K, long long stride, hipStream_t st);
template <typename T> hipError_t launch_znorm_batch(const SessDev<T> &s, int K, long long stride, hipStream_t st);
hipError_t launch_commit(DevCtl *ctl, hipStream_t st);
hipError_t launch_set_ctl(DevCtl *ctl, long long pushed, hipStream_t st);
template <typename T>
hipError_t launch_finalize_bins(const SessDev<T> &s, uint32_t metric, T *out, hipStream_t st);
hipError_t launch_copy_probe(void *dst, const void *src, int64_t n_bytes, hipStream_t st);
hipError_t launch_rmw_probe(void *buf, int64_t n_elems, hipStream_t st);
hipError_t launch_mfma_probe(int kind, int iters, float *out, double *flops, hipStream_t st);

// batch (window recompute) path, float sessions (fcx_batch.hip)
hipError_t launch_set_pushed(DevCtl *ctl, long long pushed, hipStream_t st);
hipError_t launch_batch_commit(DevCtl *ctl, long long K, hipStream_t st);
hipError_t launch_psd_batch(const SessDev<float> &s, int K, hipStream_t st);
hipError_t launch_pair_batch(const SessDev<float> &s, int K, int prec, hipStream_t st);
hipError_t launch_cor_batch(const SessDev<float> &s, int K, int prec, hipStream_t st);

// XCOR of the trial at ring slot of the push (fcx_xcor.hip): node spectra and
// suffix energies, then per pair the FFT correlation, its maximum over the
// lags and the window sum
template <typename T> hipError_t launch_xcor(const SessDev<T> &s, hipStream_t st);

// bin-chunk size of the pair kernel for a given (B, L, element size), and the
// LDS it needs
__host__ __device__ int pair_node_bytes(int L, int elem_bytes, uint32_t metrics);
__host__ __device__ int pair_chunk_bins(int B, int L, int elem_bytes, uint32_t metrics);
__host__ __device__ size_t pair_lds_bytes(int CB, int L, int elem_bytes, uint32_t metrics);
// A served session's coalesced group of nt trials stages every trial's node
// data per bin: at most pair_group_max trials fit the pair kernel's LDS with
// one bin, and pair_chunk_bins_mt bins are staged per chunk (its LDS is
// nt * pair_lds_bytes(chunk, ...) at most).
__host__ __device__ inline int pair_group_max(int L, int elem_bytes, uint32_t metrics)
{
    const int g = PAIR_LDS_BYTES / (PAIR_NODES * pair_node_bytes(L, elem_bytes, metrics));
    return g < 1 ? 1 : g;
}
__host__ __device__ inline int pair_chunk_bins_mt(int B, int L, int elem_bytes, uint32_t metrics, int nt)
{
    int cb = PAIR_LDS_BYTES / (PAIR_NODES * pair_node_bytes(L, elem_bytes, metrics) * (nt > 0 ? nt : 1));
    if (cb < 1) cb = 1;
    return cb < B ? cb : B;
}

// batched launches of the serving path (float sessions); items are
// (session index, a, b, 0) with a/b the block coordinates of the kernel
enum { FCX_B_SPECTRA = 0, FCX_B_ZNORM, FCX_B_PSD, FCX_B_COMMIT };
hipError_t launch_batched(int which, const SessDev<float> *S, const int4 *items, int n, size_t lds,
                          hipStream_t st);

// compile-time variant (class) of an FP32 session's pair update, and the
// batched pair launch over items (session, tile slice) of sessions of one class
constexpr int PAIR_CLASSES = 36;
int pair_kernel_class(const SessDev<float> &s);
hipError_t launch_batched_pair(int cls, const SessDev<float> *S, const int4 *items, int n, size_t lds,
                               hipStream_t st);

}  // namespace fcx
