"""GPU: the allocation-free entry point (dicod_solve_device_noalloc), whose
workspace lives in the library's static device scratch, against the
allocating dicod_solve_device on the same inputs, through the C ABI: two calls
in a row (the second with a smaller input, so the scratch holds the first
call's contents), each equal element by element to the allocating solve and
an eps-solution of the oracle's problem (relative objective error <= 1e-6,
max |z - z_ref| <= 1e-4 max |z_ref|, oracle stop test below eps)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS = 1e-6


@pytest.fixture(scope="module")
def dicod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_10087_amd as d
    return d


def f64(a):
    return np.asarray(a, dtype=np.float64)


def check_oracle(X, D, lam, Z, st):
    L = X.shape[1] - D.shape[2] + 1
    Zo, so, _ = oracle.lgcd(f64(X), f64(D), lam, 1e-10, max(1, L // 800))
    assert so["converged"] == 1
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    E = oracle.objective(f64(X), f64(D), Z, lam)
    assert abs(E - Eo) <= 1e-6 * Eo, (E, Eo)
    assert np.max(np.abs(Z - Zo)) <= 1e-4 * np.max(np.abs(Zo))
    mdz, _, _ = oracle.max_dz(f64(X), f64(D), Z, lam)
    assert mdz < EPS * (1 + 1e-6), mdz


@pytest.mark.parametrize("precision", [1, 0, 2])
def test_noalloc_equals_allocating_solve_two_calls(dicod, precision):
    import torch
    print(f"\ncase: no-alloc solve precision={precision}", flush=True)
    D = synth.generate(7, 25, 200, 1000, 0.007, 0.1, seed=91)[1]
    Xs = [synth.generate(7, 25, 200, T, 0.007, 0.1, seed=92 + i, D=D)[0]
          for i, T in enumerate((40_000, 12_345))]
    with dicod.Context(precision=precision, max_phases=50_000) as c:
        c.set_dictionary(D)
        for X in Xs:                      # the second call is smaller
            Xd = torch.from_numpy(X).cuda()
            L = X.shape[1] - D.shape[2] + 1
            Za = torch.full((25, L), np.nan, dtype=torch.float64, device="cuda")
            Zb = torch.full((25, L), np.nan, dtype=torch.float64, device="cuda")
            _, sa, _ = c.solve_device(Xd, -0.1, EPS, 0, Za)
            _, sb, _ = c.solve_device_noalloc(Xd, -0.1, EPS, 0, Zb)
            torch.cuda.synchronize()
            Za, Zb = Za.cpu().numpy(), Zb.cpu().numpy()
            print(f"T={X.shape[1]}: {sb['n_updates']} updates, max|dZ| {sb['max_dz']:.3g}",
                  flush=True)
            assert np.array_equal(Za, Zb)
            for k in ("n_updates", "n_phases", "nnz", "converged", "lambda", "objective",
                      "max_dz"):
                assert sa[k] == sb[k], k
            check_oracle(X, D, sb["lambda"], Zb, sb)


def test_noalloc_rejects_problems_beyond_the_scratch(dicod):
    import torch
    print("\ncase: no-alloc size limit", flush=True)
    D = synth.generate(7, 25, 200, 1000, 0.007, 0.1, seed=91)[1]
    X = np.random.default_rng(3).standard_normal((7, 600_000)).astype(np.float32)
    with dicod.Context(max_phases=50_000) as c:
        c.set_dictionary(D)
        Xd = torch.from_numpy(X).cuda()
        Z = torch.empty((25, X.shape[1] - 199), dtype=torch.float64, device="cuda")
        _, _, rc = c.solve_device_noalloc(Xd, -0.1, EPS, 0, Z, check=False)
        assert rc == dicod.DICOD_EINVAL
        assert "bytes of scratch" in dicod.dicod_last_error(c.h)
