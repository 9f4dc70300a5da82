# numpy emulation of the mixed-radix in-place Stockham inverse FFT with the
# padded LDS layout, exactly as planned for the wave kernel
import numpy as np
def xpad(m): return m + (m >> 5)
RADICES = {256: (4, 4, 4, 4), 512: (8, 8, 8), 1024: (16, 16, 4), 2048: (16, 16, 8)}
def idft_r(a):
    R = len(a)
    if R == 1: return a
    E = idft_r(a[0::2]); O = idft_r(a[1::2])
    w = np.exp(2j * np.pi * np.arange(R // 2) / R)
    return np.concatenate([E + w * O, E - w * O])
def ifft_emul(x):
    F = len(x)
    Z = np.zeros(xpad(F - 1) + 1, complex)
    for m in range(F): Z[xpad(m)] = x[m]
    tw = np.exp(-2j * np.pi * np.arange(F) / F)
    Ns = 1
    for R in RADICES[F]:
        NB = F // R; PER = NB // 64; STEP = F // (R * Ns)
        assert NB % 32 == 0 and PER >= 1
        vals = {}
        for lane in range(64):
            for q in range(PER):
                j = lane + 64 * q; k = j & (Ns - 1)
                v = []
                for r in range(R):
                    idx = xpad(j) + r * NB + ((r * NB) >> 5)
                    assert idx == xpad(j + r * NB)
                    a = Z[idx]
                    if r and Ns > 1: a = a * np.conj(tw[r * k * STEP])
                    v.append(a)
                vals[j] = idft_r(np.array(v))
        for j, y in vals.items():
            k = j & (Ns - 1); o = (j // Ns) * Ns * R + k; base = xpad(o)
            for m in range(R):
                idx = base + m * Ns + ((m * Ns) >> 5)
                assert idx == xpad(o + m * Ns), (F, R, Ns, j, m)
                Z[idx] = y[m]
        Ns *= R
    return np.array([Z[xpad(m)] for m in range(F)])
rng = np.random.default_rng(0)
for F in (256, 512, 1024, 2048):
    x = rng.standard_normal(F) + 1j * rng.standard_normal(F)
    y = ifft_emul(x)
    print(F, np.max(np.abs(y - np.fft.ifft(x) * F)))
