"""Bound on the proliferation step's parameters when the FP32 path draws its
normals in FP32 (Algorithm 1 step 4(a): theta_{j+1} = m + s L z).

The FP32 Box-Muller pair of radius r = sqrt(-2 ln u): the uniforms rounded
to FP32 (relative 2^-24) and logf, sqrtf and sincospif each within about one
unit in the last place give |dz| <= 2^-24 / r + 2^-20 r for both normals of
the pair (the radius through d(ln u) = du / u, the angle through 2 pi du and
the FP32 product).  With a factor 2 for margin, |d theta_i| <= s sum_c
|L_ic| |dz_c| (+ FP64 rounding).  TEST INFRASTRUCTURE (uses the oracle)."""
import numpy as np


def fp32_jitter_bound(oracle, prob, L, step, n_slots):
    """[n_slots][p] bounds on |theta_gpu - theta_oracle| for the slots of
    `step`, given the Cholesky factor L (p x p) the step proliferates with."""
    p = prob.p
    nb = 4 * ((p + 3) // 4)                       # whole blocks: every pair's partner
    s = np.sqrt(1.0 - prob.shrink_a ** 2)
    La = np.abs(np.asarray(L, dtype=float).reshape(p, p))
    out = np.zeros((n_slots, p))
    for n in range(n_slots):
        z = oracle.normals(prob.seed, step, n, oracle.PUR_PROLIF, nb)
        r = np.sqrt(z[0::2] ** 2 + z[1::2] ** 2)   # radius of each Box-Muller pair
        rc = np.repeat(r, 2)[:p]
        dz = 2.0 * (2.0 ** -24 / rc + 2.0 ** -20 * rc)
        out[n] = s * (La @ dz)
    return out + 1e-13
