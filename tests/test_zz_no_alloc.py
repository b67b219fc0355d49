"""The transition entry point that allocates nothing (its buffers live in the
library's static device array) against ess_transition_explicit, through the
C ABI: two calls in a row, the second with a smaller input."""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_10449_amd as E
    E.lib()
    return E


def case(rng, d, m, C, precision):
    A = rng.standard_normal((m, d)) / math.sqrt(d)
    b = rng.uniform(0.5, 1.5, m)
    npdt = np.float32 if precision == 32 else np.float64
    x = synth.random_states(rng, A, b, C, scale=0.7).astype(npdt)
    nu = rng.standard_normal((C, d)).astype(npdt)
    u = rng.uniform(size=C)
    return A, b, x, nu, u


def with_context(E, A, b, x, nu, u, precision, eps):
    s = E.Sampler(A, b, x, x.shape[0], seed=0, precision=precision, trim_eps=eps)
    out = {k: v.cpu().numpy() for k, v in s.transition_explicit(x, nu, u).items()}
    s.close()
    return out


def without_allocation(E, A, b, x, nu, u, precision, eps):
    dt = torch.float32 if precision == 32 else torch.float64
    dev = "cuda"
    m, d = A.shape
    C = x.shape[0]
    At = torch.as_tensor(A).to(dev, dt).contiguous()
    bt = torch.as_tensor(b).to(dev, torch.float64).contiguous()
    xt = torch.as_tensor(x).to(dev, dt).contiguous()
    nut = torch.as_tensor(nu).to(dev, dt).contiguous()
    ut = torch.as_tensor(u).to(dev, torch.float64).contiguous()
    out = dict(x_new=torch.empty(C, d, device=dev, dtype=dt),
               intervals=torch.zeros(C, m + 1, 2, device=dev, dtype=torch.float64),
               n_intervals=torch.zeros(C, device=dev, dtype=torch.int32),
               theta=torch.zeros(C, device=dev, dtype=torch.float64),
               rejected=torch.zeros(C, device=dev, dtype=torch.int32))
    E.ess_transition_explicit_static(d, m, C, precision, At, bt, eps, xt, nut, ut, out["x_new"],
                                     out["intervals"], out["n_intervals"], out["theta"],
                                     out["rejected"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("precision,shapes", [
    # 128 x 128 tiles and the split projections, more than 256 chains with
    # 64 x 64 tiles, then ragged and few
    (32, [(64, 2000, 1024), (1000, 2000, 300), (60, 150, 40)]),
    (64, [(65, 300, 130), (10, 20, 16)]),
])
def test_static_transition_equals_the_context_transition(E, precision, shapes):
    rng = np.random.default_rng(precision)
    eps = 1e-6 if precision == 32 else 0.0
    for d, m, C in shapes:
        print(f"[no-alloc] d={d} m={m} C={C} precision={precision}", file=sys.stderr, flush=True)
        A, b, x, nu, u = case(rng, d, m, C, precision)
        want = with_context(E, A, b, x, nu, u, precision, eps)
        got = without_allocation(E, A, b, x, nu, u, precision, eps)
        # the same kernels on the same inputs: identical results
        for k in ("x_new", "n_intervals", "theta", "rejected"):
            assert np.array_equal(got[k], want[k]), k
        for c in range(C):
            n = want["n_intervals"][c]
            assert np.array_equal(got["intervals"][c, :n], want["intervals"][c, :n]), c


def test_static_transition_rejects_what_it_cannot_hold_and_infeasible_starts(E):
    rng = np.random.default_rng(3)
    A, b, x, nu, u = case(rng, 16, 40, 8, 32)
    x_bad = x.copy()
    x_bad[5] = 50.0
    with pytest.raises(E.EssError) as ei:
        without_allocation(E, A, b, x_bad, nu, u, 32, 1e-6)
    assert ei.value.status == E.ESS_ERR_INFEASIBLE_START and "chain 5" in str(ei.value)
    with pytest.raises(E.EssError) as ei:
        E.ess_transition_explicit_static(2048, 16384, 4, 32, torch.zeros(1, device="cuda"),
                                         torch.zeros(1, device="cuda", dtype=torch.float64),
                                         0.0, torch.zeros(1, device="cuda"),
                                         torch.zeros(1, device="cuda"),
                                         torch.zeros(1, device="cuda", dtype=torch.float64),
                                         torch.zeros(1, device="cuda"))
    assert ei.value.status == E.ESS_ERR_UNSUPPORTED
    # a valid call still works after the refusals
    want = with_context(E, A, b, x, nu, u, 32, 1e-6)
    got = without_allocation(E, A, b, x, nu, u, 32, 1e-6)
    assert np.array_equal(got["x_new"], want["x_new"])
