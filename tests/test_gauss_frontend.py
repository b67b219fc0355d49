"""Appendix A front end: host Cholesky, whitening of (A, b), and the map of
samples back to x = L u + mu, against the oracle and a truncated normal."""
import math

import numpy as np
import pytest

from oracle import ess as ref_ess

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    import paper_2407_10449_amd as E
    E.lib()
    return E


def random_spd(rng, d):
    M = rng.standard_normal((d, d))
    return M @ M.T / d + 0.5 * np.eye(d)


def test_host_cholesky_matches_numpy(E):
    rng = np.random.default_rng(3)
    for d in (1, 2, 7, 64):
        S = random_spd(rng, d)
        L = E.ess_cholesky(S)
        assert np.allclose(L, np.linalg.cholesky(S), rtol=1e-12, atol=1e-12)
        assert np.allclose(L @ L.T, S, rtol=1e-12, atol=1e-12)
        assert np.all(np.triu(L, 1) == 0.0)


def test_host_cholesky_refuses_indefinite(E):
    with pytest.raises(E.EssError) as ei:
        E.ess_cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert ei.value.status == E.ESS_ERR_INVALID_ARG and "positive definite" in str(ei.value)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [32, 64])
def test_whiten_and_map_match_oracle(E, precision):
    _gpu()
    rng = np.random.default_rng(5)
    m, d = 300, 70
    A = rng.standard_normal((m, d))
    b = rng.uniform(0.5, 1.5, m)
    mu = 0.1 * rng.standard_normal(d)
    S = random_spd(rng, d)
    g = E.Gaussian(A, b, mu, Sigma=S, precision=precision)
    npdt = np.float32 if precision == 32 else np.float64
    L = np.linalg.cholesky(S)
    Aw, bw = ref_ess.whiten(A.astype(npdt).astype(np.float64), b, mu, L)
    tol = 1e-6 if precision == 32 else 1e-12
    assert np.allclose(g.A.cpu().numpy(), Aw, rtol=tol, atol=tol * np.abs(Aw).max())
    assert np.allclose(g.b.cpu().numpy(), bw, rtol=1e-12, atol=1e-12 * np.abs(bw).max())
    U = rng.standard_normal((3, 17, d)).astype(npdt)
    X = g.map(torch.as_tensor(U).cuda()).cpu().numpy()
    Xr = ref_ess.unwhiten(U.reshape(-1, d), L, mu).reshape(U.shape)
    assert np.allclose(X, Xr, rtol=tol, atol=tol * np.abs(Xr).max())


@pytest.mark.gpu
def test_truncated_normal_moments_through_the_front_end(E):
    """N(1, 2^2) truncated to [0, 3] sampled in u on the GPU and mapped back
    matches scipy.stats.truncnorm's mean and variance."""
    _gpu()
    from scipy import stats
    mu, sd, lo, hi = 1.0, 2.0, 0.0, 3.0
    g = E.Gaussian(np.array([[1.0], [-1.0]]), np.array([hi, -lo]), np.array([mu]),
                   Sigma=np.array([[sd * sd]]), precision=64)
    C, T, burn = 4096, 120, 20
    s = E.Sampler(g.A, g.b, np.zeros(1), C, seed=9, precision=64)
    trace, _ = s.run(T)
    s.close()
    x = g.map(trace[burn:]).cpu().numpy().ravel()
    ref = stats.truncnorm((lo - mu) / sd, (hi - mu) / sd, loc=mu, scale=sd)
    se = math.sqrt(ref.var() / (C * 10))
    assert abs(x.mean() - ref.mean()) < 5 * se, (x.mean(), ref.mean())
    assert abs(x.var() - ref.var()) < 0.02 * ref.var(), (x.var(), ref.var())
    assert x.min() >= lo - 1e-12 and x.max() <= hi + 1e-12


@pytest.mark.gpu
def test_correlated_samples_stay_in_the_original_polytope(E):
    """A correlated 5-d normal truncated to a random polytope: every mapped
    sample satisfies A x <= b (checked in float64 on the host)."""
    _gpu()
    rng = np.random.default_rng(8)
    d, m = 5, 12
    A = rng.standard_normal((m, d))
    mu = 0.2 * rng.standard_normal(d)
    b = A @ mu + rng.uniform(0.3, 1.0, m)
    g = E.Gaussian(A, b, mu, Sigma=random_spd(rng, d), precision=64)
    s = E.Sampler(g.A, g.b, np.zeros(d), 256, seed=2, precision=64)
    trace, _ = s.run(50)
    s.close()
    x = g.map(trace).cpu().numpy().reshape(-1, d)
    assert (x @ A.T <= b + 1e-9).all()


def test_front_end_argument_errors(E):
    """The Appendix A entry points refuse bad arguments before touching any
    device memory (host checks; runs without a GPU)."""
    lib = E.lib()
    P = E._P
    fake = P(0x1000)
    st = lib.ess_whiten(fake, fake, fake, fake, 10, 3, 16, P(0x2000), fake, None)
    assert st == E.ESS_ERR_INVALID_ARG and "precision" in E.ess_last_error()
    st = lib.ess_whiten(fake, fake, fake, fake, 0, 3, 32, P(0x2000), fake, None)
    assert st == E.ESS_ERR_INVALID_ARG
    st = lib.ess_whiten(fake, fake, fake, fake, 10, 3, 32, fake, fake, None)
    assert st == E.ESS_ERR_INVALID_ARG and "alias" in E.ess_last_error()
    st = lib.ess_whiten(None, fake, fake, fake, 10, 3, 32, P(0x2000), fake, None)
    assert st == E.ESS_ERR_INVALID_ARG
    st = lib.ess_unwhiten(fake, 0, 3, fake, fake, 32, P(0x2000), None)
    assert st == E.ESS_ERR_INVALID_ARG
    st = lib.ess_unwhiten(fake, 5, 3, fake, fake, 32, fake, None)
    assert st == E.ESS_ERR_INVALID_ARG and "alias" in E.ess_last_error()
