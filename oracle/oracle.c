/*
 * FP64 CPU oracle for the online all-to-all connectivity hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * It computes the plain definitions of the supplementary metric section
 * ("Functional Connectivity Metrics", time and frequency domain) over the
 * trials it is given, directly and in double precision:
 *
 *   spectra   X_{k,i,l}(b) = sum_n w_l[n] x_{k,i}[n] exp(-2 pi i kb n / F)
 *             (taper, zero padding to F, direct DFT at the band bins only)
 *   per trial CSD_ij = sum_l lam_l X_il conj(X_jl) / sum_l lam_l  (CSD eq.)
 *             PSD_i  = sum_l lam_l |X_il|^2       / sum_l lam_l  (PSD eq.)
 *   sums      S = sum_k CSD, P_i = sum_k PSD_i, U = sum_k CSD/|CSD|,
 *             G = sum_k sign(Im CSD), A = sum_k |Im CSD|, Q = sum_k (Im CSD)^2
 *   metrics   COH = |S|/sqrt(P_i P_j)            (COHY and COH eqs.)
 *             IMCOH = Im S / sqrt(P_i P_j)        (IMAGCOHY eq.)
 *             PLV = |U|/K                         (PLV eq.)
 *             PLI = |G|/K                         (PLI eq.)
 *             WPLI = |Im S| / A                   (WPLI eq.)
 *             USPLI = (K PLI^2 - 1)/(K - 1)       (USPLI eq.)
 *             DSWPLI = ((Im S)^2 - Q)/(A^2 - Q)   (debiased squared WPLI;
 *                       the printed "WPLI^2" is read as the debiased form)
 *   COR       mean over trials of the Pearson correlation (COR eq.)
 *   XCOR      mean over trials of the largest cross-correlation over the
 *             lags -L..L (XCOR eq., both directions; orc_xcor)
 *
 * Readings where the text is silent: sign(0) = 0; a metric whose denominator
 * is exactly zero is 0; the unit phasor of 0 is 0; USPLI and DSWPLI are NaN
 * for K < 2; the band value is the arithmetic mean of per-bin values.
 *
 * Built with -ffp-contract=off so that every product is rounded on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NMET 7 /* COH, IMCOH, PLV, PLI, WPLI, USPLI, DSWPLI */

/* exp(-2 pi i r / F) for integer r; exact where 4r is a multiple of F
 * (angles 0, pi/2, pi, 3pi/2 have exactly representable sine and cosine). */
static void twiddle(int64_t r, int64_t F, double *c, double *s)
{
    r %= F;
    if ((4 * r) % F == 0) {
        static const double cq[4] = {1.0, 0.0, -1.0, 0.0};
        static const double sq[4] = {0.0, -1.0, 0.0, 1.0};
        int q = (int)((4 * r) / F);
        *c = cq[q];
        *s = sq[q];
        return;
    }
    double th = 2.0 * M_PI * (double)r / (double)F;
    *c = cos(th);
    *s = -sin(th);
}

static double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

/*
 * Spectra of the selected nodes.
 *   x      : trial k, node i, sample n at x[k*trial_stride + i*node_stride + n]
 *   taper  : [L][M]
 *   bins   : [B] FFT bin indices (0 <= kb <= F/2)
 *   nodes  : [nn] node indices
 * Outputs (row-major [K][nn][L][B]): Xre, Xim; l1 [K][nn][L] = sum_n |w x|.
 */
void orc_spectra(const double *x, int64_t K, int64_t trial_stride, int64_t node_stride,
                 int64_t M, const double *taper, int32_t L, int64_t F,
                 const int32_t *bins, int32_t B, const int32_t *nodes, int64_t nn,
                 double *Xre, double *Xim, double *l1)
{
    double *tc = (double *)malloc(sizeof(double) * (size_t)B * (size_t)M);
    double *ts = (double *)malloc(sizeof(double) * (size_t)B * (size_t)M);
    for (int32_t b = 0; b < B; ++b)
        for (int64_t n = 0; n < M; ++n)
            twiddle((int64_t)bins[b] * n, F, &tc[b * M + n], &ts[b * M + n]);

#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < K; ++k)
        for (int64_t a = 0; a < nn; ++a) {
            const double *xi = x + k * trial_stride + (int64_t)nodes[a] * node_stride;
            for (int32_t l = 0; l < L; ++l) {
                const double *w = taper + (int64_t)l * M;
                double s1 = 0.0;
                for (int64_t n = 0; n < M; ++n) s1 += fabs(w[n] * xi[n]);
                l1[(k * nn + a) * L + l] = s1;
                for (int32_t b = 0; b < B; ++b) {
                    double re = 0.0, im = 0.0;
                    for (int64_t n = 0; n < M; ++n) {
                        double v = w[n] * xi[n];
                        re += v * tc[b * M + n];
                        im += v * ts[b * M + n];
                    }
                    int64_t o = ((k * nn + a) * L + l) * B + b;
                    Xre[o] = re;
                    Xim[o] = im;
                }
            }
        }
    free(tc);
    free(ts);
}

/*
 * Window sums and metrics for a list of pairs.
 *   Xre, Xim, l1 : as produced by orc_spectra ([K][nn][L][B], [K][nn][L])
 *   lam          : [L] taper weights
 *   pa, pb       : [np] pair endpoints as positions in the node list
 *   delta        : tie factor; trial k is a tie for (pair, bin) when
 *                  |Im CSD| <= delta * sum_l lam_l (l1_a |X_b| + l1_b |X_a|) / sum lam
 * Outputs:
 *   per_bin [np][B][7], band [np][7]  (metric order COH IMCOH PLV PLI WPLI USPLI DSWPLI)
 *   gsum [np][B] (sign sums G), ties [np][B]
 *   sums [np][B][8] (S_re, S_im, P_a, P_b, U_re, U_im, A, Q) if non-NULL
 *   aqt  [np][B][3] (A, Q, and the sum over the trials of the tie thresholds)
 *        if non-NULL: the scale on which WPLI and DSWPLI are decided by
 *        rounding alone (SI-1 WPLI and DSWPLI equations)
 */
void orc_pairs(const double *Xre, const double *Xim, const double *l1, int64_t K, int64_t nn,
               int32_t L, int32_t B, const double *lam, const int32_t *pa, const int32_t *pb,
               int64_t np, double delta, double *per_bin, double *band, int32_t *gsum,
               int32_t *ties, double *sums, double *aqt)
{
    double lsum = 0.0;
    for (int32_t l = 0; l < L; ++l) lsum += lam[l];

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pa[p], c = pb[p];
        double bandacc[NMET];
        for (int m = 0; m < NMET; ++m) bandacc[m] = 0.0;
        for (int32_t b = 0; b < B; ++b) {
            double Sre = 0, Sim = 0, Pa = 0, Pb = 0, Ure = 0, Uim = 0, A = 0, Q = 0;
            int32_t G = 0, T = 0;
            double Tsum = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double cre = 0, cim = 0, pwa = 0, pwb = 0, tau = 0;
                for (int32_t l = 0; l < L; ++l) {
                    int64_t oa = ((k * nn + a) * L + l) * B + b;
                    int64_t oc = ((k * nn + c) * L + l) * B + b;
                    double ar = Xre[oa], ai = Xim[oa], br = Xre[oc], bi = Xim[oc];
                    /* X_a conj(X_b) */
                    cre += lam[l] * (ar * br + ai * bi);
                    cim += lam[l] * (ai * br - ar * bi);
                    pwa += lam[l] * (ar * ar + ai * ai);
                    pwb += lam[l] * (br * br + bi * bi);
                    tau += lam[l] * (l1[(k * nn + a) * L + l] * sqrt(br * br + bi * bi) +
                                     l1[(k * nn + c) * L + l] * sqrt(ar * ar + ai * ai));
                }
                cre /= lsum;
                cim /= lsum;
                pwa /= lsum;
                pwb /= lsum;
                tau = delta * tau / lsum;
                Sre += cre;
                Sim += cim;
                Pa += pwa;
                Pb += pwb;
                double mag = sqrt(cre * cre + cim * cim);
                if (mag > 0.0) {
                    Ure += cre / mag;
                    Uim += cim / mag;
                }
                G += (int32_t)sgn(cim);
                if (fabs(cim) <= tau) T += 1;
                Tsum += tau;
                A += fabs(cim);
                Q += cim * cim;
            }
            double Kd = (double)K;
            double den = sqrt(Pa * Pb);
            double met[NMET];
            met[0] = den > 0.0 ? sqrt(Sre * Sre + Sim * Sim) / den : 0.0;
            met[1] = den > 0.0 ? Sim / den : 0.0;
            met[2] = K > 0 ? sqrt(Ure * Ure + Uim * Uim) / Kd : 0.0;
            double pli = K > 0 ? fabs((double)G) / Kd : 0.0;
            met[3] = pli;
            met[4] = A > 0.0 ? fabs(Sim) / A : 0.0;
            if (K < 2) {
                met[5] = NAN;
                met[6] = NAN;
            } else {
                met[5] = (Kd * pli * pli - 1.0) / (Kd - 1.0);
                double dd = A * A - Q;
                met[6] = dd != 0.0 ? (Sim * Sim - Q) / dd : 0.0;
            }
            for (int m = 0; m < NMET; ++m) {
                per_bin[(p * B + b) * NMET + m] = met[m];
                bandacc[m] += met[m];
            }
            gsum[p * B + b] = G;
            ties[p * B + b] = T;
            if (aqt) {
                double *t = aqt + (p * B + b) * 3;
                t[0] = A; t[1] = Q; t[2] = Tsum;
            }
            if (sums) {
                double *s = sums + (p * B + b) * 8;
                s[0] = Sre; s[1] = Sim; s[2] = Pa; s[3] = Pb;
                s[4] = Ure; s[5] = Uim; s[6] = A; s[7] = Q;
            }
        }
        for (int m = 0; m < NMET; ++m) band[p * NMET + m] = bandacc[m] / (double)B;
    }
}

/*
 * The incremental method on the CPU, for the throughput baseline only (its
 * networks are pinned to orc_pairs by the CPU tests): one sliding push on
 * running FP64 sums per (pair, bin) -- the new trial's per-trial terms added,
 * the evicted trial's subtracted, as the running sums of the implementation
 * section keep them -- and the band means of the seven spectral metrics of
 * the window after the push.
 *   Xn*, Xo*  : spectra of the new and of the evicted trial [nn][L][B]
 *               (orc_spectra layout for one trial); has_old = 0: no eviction
 *   psd       : [nn][B] running power sums, updated here
 *   state     : [np][B][7] running sums S_re, S_im, U_re, U_im, G, A, Q
 *   K         : trials in the window after the push
 *   band      : [np][7] band means after the push
 */
static void trial_terms(const double *Xre, const double *Xim, int64_t a, int64_t c, int32_t L, int32_t B,
                        int32_t b, const double *lam, double lsum, double *cre, double *cim)
{
    double r = 0.0, m = 0.0;
    for (int32_t l = 0; l < L; ++l) {
        int64_t oa = (a * L + l) * B + b, oc = (c * L + l) * B + b;
        r += lam[l] * (Xre[oa] * Xre[oc] + Xim[oa] * Xim[oc]);
        m += lam[l] * (Xim[oa] * Xre[oc] - Xre[oa] * Xim[oc]);
    }
    *cre = r / lsum;
    *cim = m / lsum;
}

void orc_slide(const double *Xnre, const double *Xnim, const double *Xore, const double *Xoim, int32_t has_old,
               int64_t nn, int32_t L, int32_t B, const double *lam, const int32_t *pa, const int32_t *pb,
               int64_t np, int64_t K, double *psd, double *state, double *band)
{
    double lsum = 0.0;
    for (int32_t l = 0; l < L; ++l) lsum += lam[l];
    for (int64_t a = 0; a < nn; ++a)
        for (int32_t b = 0; b < B; ++b) {
            double pn = 0.0, po = 0.0;
            for (int32_t l = 0; l < L; ++l) {
                int64_t o = (a * L + l) * B + b;
                pn += lam[l] * (Xnre[o] * Xnre[o] + Xnim[o] * Xnim[o]);
                if (has_old) po += lam[l] * (Xore[o] * Xore[o] + Xoim[o] * Xoim[o]);
            }
            psd[a * B + b] += pn / lsum;
            if (has_old) psd[a * B + b] -= po / lsum;
        }
    const double Kd = (double)K;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        int64_t a = pa[p], c = pb[p];
        double acc[NMET];
        for (int m = 0; m < NMET; ++m) acc[m] = 0.0;
        for (int32_t b = 0; b < B; ++b) {
            double *st = state + (p * B + b) * 7;
            double nr, ni;
            trial_terms(Xnre, Xnim, a, c, L, B, b, lam, lsum, &nr, &ni);
            double mag = sqrt(nr * nr + ni * ni);
            st[0] += nr;
            st[1] += ni;
            if (mag > 0.0) {
                st[2] += nr / mag;
                st[3] += ni / mag;
            }
            st[4] += sgn(ni);
            st[5] += fabs(ni);
            st[6] += ni * ni;
            if (has_old) {
                double orr, oi;
                trial_terms(Xore, Xoim, a, c, L, B, b, lam, lsum, &orr, &oi);
                double mo = sqrt(orr * orr + oi * oi);
                st[0] -= orr;
                st[1] -= oi;
                if (mo > 0.0) {
                    st[2] -= orr / mo;
                    st[3] -= oi / mo;
                }
                st[4] -= sgn(oi);
                st[5] -= fabs(oi);
                st[6] -= oi * oi;
            }
            double den = sqrt(psd[a * B + b] * psd[c * B + b]);
            double Sre = st[0], Sim = st[1], A = st[5], Q = st[6];
            acc[0] += den > 0.0 ? sqrt(Sre * Sre + Sim * Sim) / den : 0.0;
            acc[1] += den > 0.0 ? Sim / den : 0.0;
            acc[2] += sqrt(st[2] * st[2] + st[3] * st[3]) / Kd;
            double pli = fabs(st[4]) / Kd;
            acc[3] += pli;
            acc[4] += A > 0.0 ? fabs(Sim) / A : 0.0;
            if (K < 2) {
                acc[5] = NAN;
                acc[6] = NAN;
            } else {
                acc[5] += (Kd * pli * pli - 1.0) / (Kd - 1.0);
                double dd = A * A - Q;
                acc[6] += dd != 0.0 ? (Sim * Sim - Q) / dd : 0.0;
            }
        }
        for (int m = 0; m < NMET; ++m) band[p * NMET + m] = acc[m] / (double)B;
    }
}

/*
 * COR: mean over the K trials of the per-trial Pearson correlation of the two
 * nodes' samples (COR eq.); zero variance gives r = 0.
 */
void orc_cor(const double *x, int64_t K, int64_t trial_stride, int64_t node_stride, int64_t M,
             const int32_t *pi, const int32_t *pj, int64_t np, double *cor)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        double acc = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double *a = x + k * trial_stride + (int64_t)pi[p] * node_stride;
            const double *b = x + k * trial_stride + (int64_t)pj[p] * node_stride;
            double ma = 0.0, mb = 0.0;
            for (int64_t n = 0; n < M; ++n) {
                ma += a[n];
                mb += b[n];
            }
            ma /= (double)M;
            mb /= (double)M;
            double sab = 0.0, saa = 0.0, sbb = 0.0;
            for (int64_t n = 0; n < M; ++n) {
                double da = a[n] - ma, db = b[n] - mb;
                sab += da * db;
                saa += da * da;
                sbb += db * db;
            }
            double d = sqrt(saa * sbb);
            acc += d > 0.0 ? sab / d : 0.0;
        }
        cor[p] = K > 0 ? acc / (double)K : 0.0;
    }
}

/* Cross-correlation (XCOR) of the time-domain metrics section, maximised
 * over the lags as the implementation section describes, averaged over the
 * trials like COR.  For trial k, x = node pi, y = node pj, each centred by
 * its mean over the M samples (x~, y~):
 *   XCOR(tau)  = sum_{t<M-tau} x~(t+tau) y~(t)
 *                / sqrt(sum_{t<M-tau} x~(t+tau)^2 * sum_{t<M} y~(t)^2),  tau = 0..L
 *   XCOR(-tau) = the same with x and y exchanged                          tau = 1..L
 * (0 where the denominator is 0).  The trial's value is the largest of the
 * 2L+1 values; out = its mean over the K trials.  lag_last (optional) gets
 * the lag of the largest value in the last trial (first such lag from -L). */
void orc_xcor(const double *x, int64_t K, int64_t trial_stride, int64_t node_stride, int64_t M, int64_t L,
              const int32_t *pi, const int32_t *pj, int64_t np, double *out, int32_t *lag_last)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < np; ++p) {
        double *xa = (double *)malloc((size_t)M * sizeof(double));
        double *xb = (double *)malloc((size_t)M * sizeof(double));
        double acc = 0.0;
        int32_t best_lag = 0;
        for (int64_t k = 0; k < K; ++k) {
            const double *a = x + k * trial_stride + (int64_t)pi[p] * node_stride;
            const double *b = x + k * trial_stride + (int64_t)pj[p] * node_stride;
            double ma = 0.0, mb = 0.0;
            for (int64_t n = 0; n < M; ++n) {
                ma += a[n];
                mb += b[n];
            }
            ma /= (double)M;
            mb /= (double)M;
            double ea = 0.0, eb = 0.0;
            for (int64_t n = 0; n < M; ++n) {
                xa[n] = a[n] - ma;
                xb[n] = b[n] - mb;
                ea += xa[n] * xa[n];
                eb += xb[n] * xb[n];
            }
            double best = -INFINITY;
            int32_t lag = 0;
            for (int64_t s = -L; s <= L; ++s) {
                /* s >= 0: x advanced by s against y; s < 0: y advanced by -s against x */
                const double *u = s >= 0 ? xa : xb, *v = s >= 0 ? xb : xa;
                const double ev = s >= 0 ? eb : ea;
                const int64_t tau = s >= 0 ? s : -s;
                double num = 0.0, eu = 0.0;
                for (int64_t t = 0; t < M - tau; ++t) {
                    num += u[t + tau] * v[t];
                    eu += u[t + tau] * u[t + tau];
                }
                const double d = sqrt(eu * ev);
                const double r = d > 0.0 ? num / d : 0.0;
                if (r > best) {
                    best = r;
                    lag = (int32_t)s;
                }
            }
            acc += best;
            best_lag = lag;
        }
        out[p] = K > 0 ? acc / (double)K : 0.0;
        if (lag_last) lag_last[p] = best_lag;
        free(xa);
        free(xb);
    }
}

int orc_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
