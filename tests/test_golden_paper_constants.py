"""The advection-diffusion workload against the constants the paper prints
(Sec. 4, Table 3, eq. (fixedparams), Table 4), read from a text fixture:
the initial plumes, the data-generating parameters through the reading
K = [[k1, k3], [0, k2]], the diffusion entries the section states, the
difference matrix, and the observation protocol."""
import os

import numpy as np
import pytest

from paper_1411_1702_amd import inputs

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "advdiff_sec4_constants.txt")


def _fixture():
    rows = {}
    with open(FIXTURE) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.setdefault(line[0], []).append([float(v) for v in line[1:]])
    return rows


def test_plumes_are_table_3():
    plumes = np.array(_fixture()["plume"])
    assert plumes.shape == (6, 3)
    assert np.array_equal(plumes[:, 0], inputs.PLUME_GAMMA)
    assert np.array_equal(plumes[:, 1], inputs.PLUME_XC)
    assert np.array_equal(plumes[:, 2], inputs.PLUME_YC)


def test_initial_field_is_the_sum_of_the_plumes():
    plumes = np.array(_fixture()["plume"])
    n = 20
    nt = n - 1
    u = inputs.advdiff_initial(n).reshape(nt, nt)   # u[iy, ix]
    for iy, ix in ((0, 0), (15, 4), (7, 7), (9, 13), (18, 2)):
        x, y = ix / nt, iy / nt
        want = sum(np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2 * g * g)) / (g * np.sqrt(2 * np.pi))
                   for g, xc, yc in plumes)
        assert u[iy, ix] == pytest.approx(want, rel=1e-14)


def test_parameters_are_eq_fixedparams():
    f = _fixture()
    K = np.array(f["K"][0]).reshape(2, 2)
    c = np.array(f["c"][0])
    assert K[1, 0] == 0.0
    k1, k3, k2 = K[0, 0], K[0, 1], K[1, 1]
    assert inputs.ADVDIFF_THETA == (k1, k2, k3, c[0], c[1])
    # the diffusion entries Sec. 4 states, d11 = k1^2, d12 = k1 k3,
    # d22 = k2^2 + k3^2, are those of K^T K
    D = np.array(f["D"][0]).reshape(2, 2)
    assert np.array_equal(K.T @ K, D)
    assert (D[0, 0], D[0, 1], D[1, 1]) == (k1 ** 2, k1 * k3, k2 ** 2 + k3 ** 2)


def test_operator_uses_the_printed_difference_matrix_and_diffusion():
    """L = -(d11 B1^T B1 + d12 (B1^T B2 + B2^T B1) + d22 B2^T B2) + c1 B1 + c2 B2
    with B1 = I (x) l, B2 = l (x) I and l the periodic difference matrix
    (1 on the diagonal, -1 below it and in the top right corner)."""
    f = _fixture()
    nt = 5
    ell = np.eye(nt) - np.eye(nt, k=-1)
    ell[0, nt - 1] = -1.0
    B1, B2 = np.kron(np.eye(nt), ell), np.kron(ell, np.eye(nt))
    D = np.array(f["D"][0]).reshape(2, 2)
    c = np.array(f["c"][0])
    want = -(D[0, 0] * B1.T @ B1 + D[0, 1] * (B1.T @ B2 + B2.T @ B1) + D[1, 1] * B2.T @ B2) + c[0] * B1 + c[1] * B2
    got = inputs._advdiff_operator(nt, inputs.ADVDIFF_THETA).toarray()
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_observation_protocol():
    f = _fixture()
    sites, T, div = int(f["sites"][0][0]), int(f["observations"][0][0]), f["noise_divisor"][0][0]
    prob = inputs.advdiff(64, T, seed=0, n=20, sites=sites)
    assert prob.m == sites and len(prob.times) == T
    assert np.array_equal(prob.times, np.arange(1, T + 1, dtype=float))
    assert len(np.unique(prob.obs_index)) == sites
    u0 = inputs.advdiff_initial(20)
    assert np.allclose(prob.sigma, np.abs(u0[prob.obs_index]).max() / div)
    # Table 4's filter settings: BDF2, h = 0.1 per time unit, N = 5000, n = 20 and 40
    h, N = f["h"][0][0], int(f["particles"][0][0])
    for n in (int(v) for v in f["sizes"][0]):
        cfg = inputs.advdiff(N, 2, seed=0, n=n)
        assert cfg.order == 2 and cfg.lmm == 0 and cfg.n_particles == N
        assert (cfg.times[0] - cfg.t0) / cfg.substeps == pytest.approx(h)
        assert cfg.d == (n - 1) ** 2
