"""GPU: Algorithm 2 without phase barriers (schedule ASYNC) and hypothesis H1.

The free-running schedule's iterates depend on timing (concurrent updates of
adjacent segments may interfere, Sec. 3), so parity is at the result level:
every returned Z is an eps-solution against the FP64 oracle run to
eps_ref = 1e-10 -- relative objective error <= 1e-6, max |z - z_ref| <=
1e-4 max |z_ref|, and the oracle's own stop test of the returned Z below eps.
The trace of a free-running solve is checked for consistency (one record per
applied update, numbered in selection order) and the interfering pairs it
reveals satisfy the Prop. A.2 identity of the objective.
"""
import bisect

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


def check(X, D, lam, Z, st):
    Zo, so, _ = oracle.lgcd(f64(X), f64(D), lam, 1e-10, 8)
    assert so["converged"] == 1
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    E = oracle.objective(f64(X), f64(D), Z, lam)
    assert abs(E - Eo) <= 1e-6 * Eo, (E, Eo)
    assert abs(st["objective"] - E) <= 1e-9 * E
    assert np.max(np.abs(Z - Zo)) <= 1e-4 * np.max(np.abs(Zo))
    assert st["converged"] == 1 and st["max_dz"] < EPS
    mdz, _, _ = oracle.max_dz(f64(X), f64(D), Z, lam)
    assert mdz < EPS * (1 + 1e-6), mdz


@pytest.mark.parametrize("case", ["random", "paper", "shifted", "two_channel"])
def test_check_h1_matches_oracle(dicod, case):
    rng = np.random.default_rng(4)
    if case == "random":
        D = rng.standard_normal((6, 3, 11))
    elif case == "paper":
        D = synth.dictionary(np.random.Generator(np.random.PCG64(2)), 25, 7, 200)
    elif case == "shifted":   # an atom and its one-sample shift: the bound 1 is reached
        D = np.array([[[0.6, -0.8, 0.0]], [[0.0, 0.6, -0.8]]])
    else:
        D = np.array([[[1.0, 0.0], [0.0, 1.0]], [[0.0, 1.0], [1.0, 0.0]]])
    D = D.astype(np.float32)
    with dicod.Context() as c:
        c.set_dictionary(D)
        r, holds = c.check_h1()
    ro = oracle.h1_ratio(f64(D))
    print(f"\ncase {case}: H1 ratio gpu {r:.15f} oracle {ro:.15f}", flush=True)
    assert abs(r - ro) <= 1e-12
    assert holds == (ro < 1.0)
    if case == "shifted":
        assert not holds
    if case == "two_channel":
        assert abs(r - 0.5) <= 1e-15


# (K, P, W, T, M): team shapes of 1, 2 and 4 waves, and the paper's atoms
CASES = [
    (5, 1, 32, 4096, 64),
    (25, 7, 64, 20000, 312),
    (3, 2, 40, 6000, 60),
    (25, 7, 200, 30000, 149),
    (25, 7, 200, 150000, 0),
]


@pytest.mark.parametrize("K,P,W,T,M", CASES)
@pytest.mark.parametrize("policy", ["fp32", "mixed_float_only"])
def test_async_matches_oracle(dicod, K, P, W, T, M, policy):
    print(f"\ncase: async K={K} P={P} W={W} T={T} M={M} {policy}", flush=True)
    X, D, _ = synth.generate(P, K, W, T, 0.007, 0.1, seed=5 * T + K)
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    cfg = dict(schedule=dicod.DICOD_SCHED_ASYNC, max_phases=50_000)
    if policy != "fp32":
        cfg.update(precision=dicod.DICOD_PREC_MIXED, fp64_polish_after=0)
    with dicod.Context(**cfg) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=M, D=D)
    print(f"gpu: {st['n_updates']} updates, {st['n_phases']} phases, rounds "
          f"{st['round_updates']} states {st['round_state']}", flush=True)
    assert st["round_state"][0] & 8 and st["round_state"][0] & 4
    if policy != "fp32":
        assert st["polished_fp64"] == 0
    assert abs(st["lambda"] - lam) <= 1e-12 * lam
    check(X, D, lam, Z, st)


def test_async_batch_matches_oracle_per_signal(dicod):
    import torch
    rng = np.random.default_rng(6)
    D = synth.dictionary(np.random.Generator(np.random.PCG64(3)), 25, 7, 64).astype(np.float32)
    Ts = [int(t) for t in rng.integers(3000, 20000, size=4)]
    Xs = [synth.generate_fast(7, 25, 64, T, 0.005, 0.1, 200 + i, D) for i, T in enumerate(Ts)]
    K, P, W = D.shape
    Ls = [T - W + 1 for T in Ts]
    x_off = np.concatenate([[0], np.cumsum([P * T for T in Ts])[:-1]]).astype(np.int64)
    z_off = np.concatenate([[0], np.cumsum([K * L for L in Ls])[:-1]]).astype(np.int64)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.concatenate([x.ravel() for x in Xs])).to(dev)
    Zb = torch.zeros(int(sum(K * L for L in Ls)), dtype=torch.float64, device=dev)
    with dicod.Context(schedule=dicod.DICOD_SCHED_ASYNC, max_phases=50_000) as c:
        c.set_dictionary(D)
        sts = c.solve_batch_device(Xd, np.array(Ts), x_off, np.full(len(Ts), -0.1), EPS, None,
                                   Zb, z_off)
    Zh = Zb.cpu().numpy()
    for i, (X, T, L) in enumerate(zip(Xs, Ts, Ls)):
        print(f"signal {i}: T={T}, {sts[i]['n_updates']} updates", flush=True)
        assert sts[i]["round_state"][0] & 8
        check(X, D, sts[i]["lambda"], Zh[z_off[i]:z_off[i] + K * L].reshape(K, L), sts[i])


def interfering_pairs(tr, W):
    """Pairs (u, v) of updates where v, in the segment that received u's
    record, was selected after u and before that segment applied u's record
    (so v's candidate ignored u), with |t_u - t_v| < W."""
    upd = tr[tr["k0"] >= 0]
    app = tr[tr["k0"] < 0]
    by_seq = {int(r["n_local"]): r for r in upd}
    per_seg = {}
    for r in upd:
        per_seg.setdefault(int(r["seg"]), []).append((int(r["n_local"]), r))
    for v in per_seg.values():
        v.sort(key=lambda x: x[0])
    pairs = []
    for a in app:
        u = by_seq.get(int(a["n_local"]))
        if u is None:
            continue
        lst = per_seg.get(int(a["seg"]), [])
        keys = [s for s, _ in lst]
        lo = bisect.bisect_right(keys, int(a["n_local"]))
        hi = bisect.bisect_left(keys, int(a["t0"]))
        for _, v in lst[lo:hi]:
            if abs(int(v["t0"]) - int(u["t0"])) < W:
                pairs.append((u, v))
    return upd, app, pairs


def test_async_trace_and_prop_a2_on_interfering_pairs(dicod):
    """A traced free-running solve with segments of W - 1 positions (so most
    updates reach a neighbour): one record per update, numbers unique; every
    applied record names a logged update of an adjacent segment; and for the
    interfering pairs found, E(Z + a + b) - E(Z + a) - E(Z + b) + E(Z) equals
    S_{k_u,k_v}[t_u - t_v] d_u d_v (Prop. A.2's interference term) at the
    returned Z."""
    P, K, W, T = 7, 25, 64, 12000
    X, D, _ = synth.generate(P, K, W, T, 0.01, 0.1, seed=17)
    L = T - W + 1
    M = L // (W - 1)
    with dicod.Context(schedule=dicod.DICOD_SCHED_ASYNC, max_phases=50_000,
                       trace_capacity=2_000_000, fp64_polish_after=0) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=M, D=D)
        tr = c.trace()
    upd, app, pairs = interfering_pairs(tr, W)
    print(f"\n{st['n_updates']} updates, {len(upd)} update records, {len(app)} applied "
          f"records, {len(pairs)} interfering pairs", flush=True)
    assert len(upd) == st["n_updates"]
    seqs = upd["n_local"].astype(np.int64)
    assert len(np.unique(seqs)) == len(seqs)
    # every applied record comes from a logged update of an adjacent segment
    seg_of = {int(r["n_local"]): int(r["seg"]) for r in upd}
    for a in app:
        assert abs(seg_of[int(a["n_local"])] - int(a["seg"])) == 1
        assert int(a["t0"]) >= int(a["n_local"])     # applied after it was selected
    check(X, D, st["lambda"], Z, st)
    # Prop. A.2 identity on up to 25 interfering pairs
    S = oracle.s_table(f64(D))
    lam = st["lambda"]
    E0 = oracle.objective(f64(X), f64(D), Z, lam)
    n_chk = 0
    for u, v in pairs[:25]:
        ku, tu, du = int(u["k0"]), int(u["t0"]), float(u["delta"])
        kv, tv, dv = int(v["k0"]), int(v["t0"]), float(v["delta"])
        if (ku, tu) == (kv, tv):
            continue
        Za, Zb, Zab = Z.copy(), Z.copy(), Z.copy()
        Za[ku, tu] += du
        Zb[kv, tv] += dv
        Zab[ku, tu] += du
        Zab[kv, tv] += dv
        lhs = (oracle.objective(f64(X), f64(D), Zab, lam) - oracle.objective(f64(X), f64(D), Za, lam)
               - oracle.objective(f64(X), f64(D), Zb, lam) + E0)
        rhs = S[ku, kv, tu - tv + W - 1] * du * dv
        tol = 1e-12 * max(1.0, abs(E0))       # cancellation of four objectives
        assert abs(lhs - rhs) <= tol + 1e-9 * abs(rhs), (lhs, rhs, tol)
        n_chk += abs(rhs) > 100 * tol
    print(f"Prop. A.2 identity checked on {n_chk} pairs with a term above the rounding",
          flush=True)
    assert n_chk >= 5


def test_async_unsupported_configurations(dicod):
    X, D, _ = synth.generate(1, 5, 32, 4096, 0.01, 0.1, seed=1)
    with dicod.Context(schedule=dicod.DICOD_SCHED_ASYNC,
                       precision=dicod.DICOD_PREC_FP64) as c:
        with pytest.raises(dicod.DicodError) as e:
            c.solve(X, -0.1, EPS, n_seg=64, D=D)
        assert e.value.code == dicod.DICOD_ENOTSUP
    with dicod.Context(schedule=dicod.DICOD_SCHED_ASYNC) as c:
        with pytest.raises(dicod.DicodError) as e:   # segments of 1016 positions
            c.solve(X, -0.1, EPS, n_seg=4, D=D)
        assert e.value.code == dicod.DICOD_ENOTSUP
