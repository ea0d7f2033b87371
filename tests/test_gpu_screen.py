"""GPU: duality gap and Gap Safe screening of the returned solution.

The library reports, for every solve, the duality gap of the returned Z with
the rescaled residual as dual point (an upper bound of E(Z) - E(Z*)), and
with screen = 1 the number of coordinates the Gap Safe sphere rule proves
zero.  Both are held to the oracle's computation from its definitions at the
same Z; the count may differ only on coordinates whose rule value rounds
across 1.
"""
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


@pytest.mark.parametrize("K,P,W,T,policy,norms", [
    (5, 1, 32, 4096, 1, "unit"),
    (25, 7, 64, 20000, 1, "scaled"),
    (25, 7, 200, 30000, 0, "unit"),
    (25, 7, 200, 30000, 2, "unit"),
])
def test_gap_and_screening_match_oracle(dicod, K, P, W, T, policy, norms):
    print(f"\ncase: gap K={K} P={P} W={W} T={T} precision={policy} {norms}", flush=True)
    X, D, _ = synth.generate(P, K, W, T, 0.007, 0.1, seed=7 * T + K)
    if norms == "scaled":
        rng = np.random.default_rng(K)
        D = (f64(D) * rng.uniform(0.3, 3.0, size=K)[:, None, None]).astype(np.float32)
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    with dicod.Context(precision=policy, screen=1, max_phases=50_000) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    g_o, r_o, mask = oracle.gap_safe(f64(X), f64(D), Z, lam)
    E = oracle.objective(f64(X), f64(D), Z, lam)
    Zo, _, _ = oracle.lgcd(f64(X), f64(D), lam, 1e-10, 8)
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    n_o = int(mask.sum())
    print(f"gap gpu {st['duality_gap']:.6g} oracle {g_o:.6g}; screened gpu {st['n_screened']} "
          f"oracle {n_o} of {Z.size}; E - E* = {E - Eo:.3g}", flush=True)
    assert abs(st["duality_gap"] - g_o) <= 1e-10 * E + 1e-6 * g_o
    assert E - Eo <= st["duality_gap"] * (1 + 1e-6) + 1e-9 * E     # weak duality
    assert abs(st["n_screened"] - n_o) <= max(2, Z.size // 100_000)
    assert not np.any(Zo[mask] != 0)        # the rule is safe at the returned Z
    assert n_o > 0.5 * np.count_nonzero(Zo == 0)


def test_gap_without_screening_and_in_batches(dicod):
    """screen = 0: the gap is still reported (n_screened = -1); a batch reports
    each signal's own gap."""
    import torch
    D = synth.dictionary(np.random.Generator(np.random.PCG64(5)), 25, 7, 64).astype(np.float32)
    Ts = [5000, 12000, 8000]
    Xs = [synth.generate_fast(7, 25, 64, T, 0.005, 0.1, 300 + i, D) for i, T in enumerate(Ts)]
    K, P, W = D.shape
    Ls = [T - W + 1 for T in Ts]
    x_off = np.concatenate([[0], np.cumsum([P * T for T in Ts])[:-1]]).astype(np.int64)
    z_off = np.concatenate([[0], np.cumsum([K * L for L in Ls])[:-1]]).astype(np.int64)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.concatenate([x.ravel() for x in Xs])).to(dev)
    Zb = torch.zeros(int(sum(K * L for L in Ls)), dtype=torch.float64, device=dev)
    with dicod.Context(max_phases=50_000) as c:
        c.set_dictionary(D)
        sts = c.solve_batch_device(Xd, np.array(Ts), x_off, np.full(3, -0.1), EPS, None, Zb,
                                   z_off)
    Zh = Zb.cpu().numpy()
    for i, (X, L) in enumerate(zip(Xs, Ls)):
        Z = Zh[z_off[i]:z_off[i] + K * L].reshape(K, L)
        g_o, _, _ = oracle.gap_safe(f64(X), f64(D), Z, sts[i]["lambda"])
        E = oracle.objective(f64(X), f64(D), Z, sts[i]["lambda"])
        assert sts[i]["n_screened"] == -1
        assert abs(sts[i]["duality_gap"] - g_o) <= 1e-10 * E + 1e-6 * g_o
