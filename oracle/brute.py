"""Pure-Python brute force for tiny inputs (test infrastructure only).

Written independently of oracle.c, straight from the definitions: a textbook
DFT with complex exponentials, per-trial CSD/PSD, and explicit loops over
trials for every sum.  USPLI and DSWPLI are also computed in Vinck's
pairwise form (sums over trial pairs j != k), which agrees with the closed
forms used by the oracle whenever no sign is zero.
"""
from __future__ import annotations

import cmath
import math


def _exp_neg(k: int, n: int, F: int) -> complex:
    # exp(-2 pi i k n / F); the angles that are multiples of pi/2 are exact
    r = (k * n) % F
    if (4 * r) % F == 0:
        return [1 + 0j, -1j, -1 + 0j, 1j][(4 * r) // F]
    return cmath.exp(-2j * math.pi * r / F)


def dft(xs, w, k, F):
    return sum(w[n] * xs[n] * _exp_neg(k, n, F) for n in range(len(xs)))


def sign(v: float) -> int:
    return 1 if v > 0 else (-1 if v < 0 else 0)


def pair_metrics(trials, i, j, w_list, lam, bins, F):
    """trials: nested lists [K][N][M]; w_list: tapers [L][M]; lam: weights.
    Returns per-bin dicts with every metric plus the Vinck pairwise forms."""
    K = len(trials)
    out = []
    lsum = sum(lam)
    for kb in bins:
        csd, psd_i, psd_j = [], [], []
        for k in range(K):
            c = 0j
            pi_ = 0.0
            pj_ = 0.0
            for w, lm in zip(w_list, lam):
                Xi = dft(trials[k][i], w, kb, F)
                Xj = dft(trials[k][j], w, kb, F)
                c += lm * Xi * Xj.conjugate()
                pi_ += lm * abs(Xi) ** 2
                pj_ += lm * abs(Xj) ** 2
            csd.append(c / lsum)
            psd_i.append(pi_ / lsum)
            psd_j.append(pj_ / lsum)
        mean_csd = sum(csd) / K
        den = math.sqrt((sum(psd_i) / K) * (sum(psd_j) / K))
        cohy = mean_csd / den if den > 0 else 0j
        phasors = [c / abs(c) if abs(c) > 0 else 0j for c in csd]
        ims = [c.imag for c in csd]
        signs = [sign(v) for v in ims]
        pli = abs(sum(signs) / K)
        mean_abs = sum(abs(v) for v in ims) / K
        wpli = abs(sum(ims) / K) / mean_abs if mean_abs > 0 else 0.0
        if K >= 2:
            uspli = (K * pli * pli - 1.0) / (K - 1.0)
            num = 0.0
            den2 = 0.0
            s_pair = 0
            for a in range(K):
                for b in range(K):
                    if a != b:
                        num += ims[a] * ims[b]
                        den2 += abs(ims[a]) * abs(ims[b])
                        s_pair += signs[a] * signs[b]
            dswpli = num / den2 if den2 != 0 else 0.0
            uspli_pairwise = s_pair / (K * (K - 1.0))
        else:
            uspli = dswpli = uspli_pairwise = float("nan")
        out.append(dict(coh=abs(cohy), imcoh=cohy.imag, plv=abs(sum(phasors) / K), pli=pli,
                        wpli=wpli, uspli=uspli, dswpli=dswpli, uspli_pairwise=uspli_pairwise,
                        G=sum(signs), any_zero_sign=any(s == 0 for s in signs)))
    return out


def pearson(a, b):
    M = len(a)
    ma = sum(a) / M
    mb = sum(b) / M
    sab = sum((a[n] - ma) * (b[n] - mb) for n in range(M))
    saa = sum((a[n] - ma) ** 2 for n in range(M))
    sbb = sum((b[n] - mb) ** 2 for n in range(M))
    d = math.sqrt(saa * sbb)
    return sab / d if d > 0 else 0.0


def cor(trials, i, j):
    return sum(pearson(t[i], t[j]) for t in trials) / len(trials)
