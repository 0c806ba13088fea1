"""Coefficients of the Chebyshev expansion of erfcx(x) = e^{x^2} erfc(x), x >= 0,
in t = (x - K)/(x + K), used by the real-space kernels (kernels.hip,
kErfcxCheb).  The map x -> t takes [0, inf) onto [-1, 1) (the variable of
Schonfelder's Chebyshev expansions of the error functions, Math. Comp. 32
(1978)); erfcx is analytic in t there, so the series converges geometrically.
The coefficients come from the discrete cosine transform of erfcx at 200
Chebyshev nodes in 40-digit arithmetic (mpmath); the script also reports the
largest relative error of the double-precision Clenshaw sum against mpmath
on a grid of x in [0, 40].  Run: python gen_erfcx.py"""
import mpmath as mp
import numpy as np

K = 3.0
N = 22       # highest order kept
M = 200      # nodes
mp.mp.dps = 40


def erfcx(x):
    x = mp.mpf(x)
    return mp.erfc(x) * mp.exp(x * x)


def coefficients():
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / M) for k in range(M)]
    vals = [erfcx(K * (1 + t) / (1 - t)) for t in nodes]
    c = []
    for n in range(N + 1):
        s = mp.fsum(vals[k] * mp.cos(mp.pi * n * (k + mp.mpf(1) / 2) / M) for k in range(M))
        c.append(2 * s / M)
    c[0] /= 2
    return [float(v) for v in c]


def clenshaw(c, x):
    t = (x - K) / (x + K)
    b1 = b2 = 0.0
    for cn in reversed(c[1:]):
        b1, b2 = 2.0 * t * b1 - b2 + cn, b1
    return t * b1 - b2 + c[0]


if __name__ == "__main__":
    c = coefficients()
    worst = 0.0
    for x in np.concatenate([np.linspace(0.0, 8.0, 8001), np.linspace(8.0, 40.0, 2001)]):
        ref = float(erfcx(x))
        worst = max(worst, abs(clenshaw(c, float(x)) / ref - 1.0))
    print(f"// K = {K}, orders 0..{N}; largest relative error on [0, 40]: {worst:.2e}")
    for i in range(0, len(c), 3):
        print("    " + " ".join(f"{v:+.17e}," for v in c[i:i + 3]))
