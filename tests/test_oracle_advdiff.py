"""Pins of the oracle's advection-diffusion model (Sec. 4): the assembled
operator against its Fourier symbol (circulant diagonalisation, derived
independently of the assembly), against the continuous operator on a smooth
wave, mass conservation, transposition symmetry, BDF (and the SDIRK start-up)
against the same recurrences run mode by mode with numpy's FFT, convergence
to the matrix exponential, and a short filter run."""
import numpy as np
import pytest
import scipy.linalg

from paper_1411_1702_amd import inputs

MODEL = 3
THETA_TRUE = np.array(inputs.ADVDIFF_THETA)


def _symbol(nt, theta):
    """lambda[p, q] for the Fourier mode exp(2 pi i (p iy + q ix) / nt): the
    periodic backward difference multiplies it by mu = 1 - exp(-2 pi i k / nt)
    along its axis, and its transpose by conj(mu)."""
    k1, k2, k3, c1, c2 = theta
    mu = 1.0 - np.exp(-2j * np.pi * np.arange(nt) / nt)
    mx = mu[None, :]          # along ix (q)
    my = mu[:, None]          # along iy (p)
    return (-(k1 * k1 * np.abs(mx) ** 2 + k1 * k3 * (np.conj(mx) * my + np.conj(my) * mx)
              + (k2 * k2 + k3 * k3) * np.abs(my) ** 2) + c1 * mx + c2 * my)


def _rhs(oracle, x, theta, nt):
    return oracle.rhs(MODEL, x, theta, mc=np.array([float(nt)]))


@pytest.mark.parametrize("nt", [5, 8])
def test_operator_fourier_symbol(oracle, nt):
    theta = np.array([1.3, 0.7, -0.4, 0.9, -1.6])
    d = nt * nt
    x = np.random.default_rng(nt).standard_normal(d)
    f, J = _rhs(oracle, x, theta, nt)
    assert np.allclose(f, J @ x, rtol=0, atol=1e-12 * np.abs(f).max())
    lam = _symbol(nt, theta)
    iy, ix = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    for p in range(nt):
        for q in range(nt):
            v = np.exp(2j * np.pi * (p * iy + q * ix) / nt).ravel()
            assert np.allclose(J @ v, lam[p, q] * v, rtol=0, atol=1e-12 * (1 + abs(lam[p, q])))


def test_operator_matches_pde_on_smooth_wave(oracle):
    # u = cos(a ix + b iy) with (a, b) = 2 pi (1, -1) / nt: div(D grad u) =
    # -(phi^T D phi) u and c . grad u = -(c . phi) sin(.), in grid units, with
    # D = K^T K, K = [[k1, k3], [0, k2]].  Absolute truncation errors: O(phi^4)
    # for the second differences, O(phi^2) for the advection's one-sided ones.
    def errors(nt, c):
        k1, k2, k3 = 2.0, 1.5, -1.0
        Dm = np.array([[k1, 0.0], [k3, k2]]) @ np.array([[k1, k3], [0.0, k2]])
        a, b = 2 * np.pi / nt, -2 * np.pi / nt
        iy, ix = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
        arg = a * ix + b * iy
        f, _ = oracle.rhs(MODEL, np.cos(arg).ravel(), np.array([k1, k2, k3, c[0], c[1]]),
                          mc=np.array([float(nt)]), d=nt * nt)
        phi = np.array([a, b])
        want = (-(phi @ Dm @ phi) * np.cos(arg) - (c[0] * a + c[1] * b) * np.sin(arg)).ravel()
        return np.abs(f - want).max(), np.abs(want).max()

    (e1, _), (e2, w2) = errors(18, (0.0, 0.0)), errors(36, (0.0, 0.0))
    assert e2 < 0.01 * w2 and 14.5 < e1 / e2 < 17.5
    (e1, _), (e2, w2) = errors(18, (0.8, 0.5)), errors(36, (0.8, 0.5))
    assert e2 < 0.08 * w2 and 3.5 < e1 / e2 < 6.5     # phi^3 terms still visible at nt = 18


def test_mass_is_conserved(oracle):
    nt = 8
    prob = inputs.advdiff(16, 2, n=nt + 1)
    f, _ = _rhs(oracle, prob.x0, THETA_TRUE, nt)
    assert abs(f.sum()) < 1e-12 * np.abs(f).max()
    for lmm, k in ((0, 2), (0, 3), (1, 1), (2, 3)):
        x, g, _ = oracle.psi(MODEL, prob.x0, THETA_TRUE, 0.1, 10, k, lte=True, mc=prob.model_consts,
                             floor=prob.state_floor, lmm=lmm)
        assert x.sum() == pytest.approx(prob.x0.sum(), rel=1e-12)


def test_transposition_symmetry(oracle):
    # D = k^2 I and c1 = c2: the operator commutes with swapping x and y
    nt = 7
    theta = np.array([1.1, 1.1, 0.0, 0.6, 0.6])
    x0 = np.random.default_rng(1).uniform(0.5, 1.5, (nt, nt))
    a, ga, _ = oracle.psi(MODEL, x0.ravel(), theta, 0.2, 5, 2, lte=True, mc=np.array([float(nt)]))
    b, gb, _ = oracle.psi(MODEL, x0.T.ravel(), theta, 0.2, 5, 2, lte=True, mc=np.array([float(nt)]))
    assert np.allclose(a.reshape(nt, nt).T.ravel(), b, rtol=1e-13, atol=0)
    assert np.allclose(ga.reshape(nt, nt).T.ravel(), gb, rtol=1e-10, atol=0)


_ALPHA = {1: [1.0, -1.0], 2: [1.0, -4 / 3, 1 / 3], 3: [1.0, -18 / 11, 9 / 11, -2 / 11]}
_BETA = {1: 1.0, 2: 2 / 3, 3: 6 / 11}
_ERRC = {1: 1 / 2, 2: 2 / 9, 3: 3 / 22}
_EXTRAP = {1: [2, -1], 2: [3, -3, 1], 3: [4, -6, 4, -1]}


def _fourier_psi(nt, theta, x0, h, M, k, sdirk_A=None):
    """BDFk with the restart ramp (and optionally the SDIRK start-up), mode by
    mode: every step is a scalar division in Fourier space; the local-error
    estimate (the Milne difference divided by 1 - h beta lambda, twice at the
    first step) is brought back to the grid with the inverse FFT and squared."""
    lam = _symbol(nt, theta)
    H = [np.fft.fft2(x0.reshape(nt, nt))]     # H[0] = x_{m-1}
    gam = np.zeros((nt, nt))
    for m in range(1, M + 1):
        avail = len(H) - 1
        q = max(1, min(k, avail))
        if avail == 0:
            xp, cstar = H[0] * (1 + h * lam), 0.5
        else:
            xp, cstar = sum(w * H[r] for r, w in enumerate(_EXTRAP[q])), 1.0
        den = 1 - h * _BETA[q] * lam
        if sdirk_A is not None and avail < k - 1:
            F = []
            for s in range(len(sdirk_A)):
                ps = H[0] + h * sum(sdirk_A[s][j] * F[j] for j in range(s))
                Y = ps / (1 - h * sdirk_A[s][s] * lam)
                F.append(lam * Y)
            x = Y
        else:
            psi = -sum(_ALPHA[q][r] * H[r - 1] for r in range(1, q + 1))
            x = psi / den
        kap = _ERRC[q] / (cstar + _ERRC[q])
        # the first step's Euler comparison passes the filter twice
        e = np.real(np.fft.ifft2(kap * (x - xp) / (den * den if avail == 0 else den)))
        gam += e * e
        H = [x] + H[:3]
    return np.real(np.fft.ifft2(H[0])).ravel(), gam.ravel()


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("sd", [False, True])
def test_bdf_equals_fourier_recurrence(oracle, k, sd):
    if sd and k == 1:
        pytest.skip("no start-up at k = 1")
    nt = 8
    prob = inputs.advdiff(16, 2, n=nt + 1)
    rng = np.random.default_rng(k)
    theta = THETA_TRUE + 0.3 * rng.standard_normal(5)
    x0 = prob.x0 * (1 + 0.05 * rng.standard_normal(prob.d))
    h, M = 0.1, 10
    xo, go, st = oracle.psi(MODEL, x0, theta, h, M, k, lte=True, mc=prob.model_consts,
                            floor=prob.state_floor, lmm=2 if sd else 0)
    A = oracle.sdirk(k)[0] if sd else None
    xf, gf = _fourier_psi(nt, theta, x0, h, M, k, A)
    assert np.abs(xo - xf).max() < 1e-11 * np.abs(xf).max()
    assert np.abs(go - gf).max() < 1e-9 * gf.max()
    assert st["newton_fails"] == 0


def test_convergence_to_matrix_exponential(oracle):
    nt = 8
    prob = inputs.advdiff(16, 2, n=nt + 1)
    _, J = _rhs(oracle, prob.x0, THETA_TRUE, nt)
    # the exponential of the operator is also what generates the data
    assert np.allclose(scipy.linalg.expm(1.0 * J) @ prob.x0, prob.x_true[0], rtol=1e-10, atol=1e-12)

    # orders in the asymptotic range: a weakly diffusive operator (h |lambda| < 0.2)
    theta = np.array([1.0, 0.8, 0.5, 0.6, -0.4])
    _, J = _rhs(oracle, prob.x0, theta, nt)
    exact = scipy.linalg.expm(0.5 * J) @ prob.x0

    def err(k, M, lmm=0):
        x, _, _ = oracle.psi(MODEL, prob.x0, theta, 0.5 / M, M, k, mc=prob.model_consts,
                             floor=prob.state_floor, lmm=lmm)
        return np.abs(x - exact).max()

    for k, lmm, order in ((1, 0, 1), (2, 0, 2), (3, 2, 3)):
        e = [err(k, M, lmm) for M in (40, 80, 160)]
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(rates - order) < 0.15), (k, lmm, rates)


def test_filter_runs_and_tracks_the_field(oracle):
    prob = inputs.advdiff(200, 3, seed=1, n=7)
    F = oracle.Filter(prob)
    for j in range(prob.T):
        out = F.step(prob.times[j], prob.y[j], prob.sigma[j])
        assert out["status"] == 0
        assert out["ess"] > 10
        assert out["newton_fails"] == 0
        err = np.abs(out["state_mean"][prob.obs_index] - prob.x_true[j, prob.obs_index])
        assert np.all(err < 5 * prob.sigma[j])
    mean, cov = F.moments()
    assert np.all(np.sqrt(np.diag(cov)) < 1.5 * prob.prior_sd)
