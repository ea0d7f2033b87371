"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Tolerances (floating point; the stop threshold is eps = 1e-6):
  * S table and beta at Z = 0 are double-precision MFMA contractions of the
    same float inputs: |gpu - oracle| <= 1e-12 * max(1, scale).
  * FP64 policy, even/odd schedule: the sequence of updates (phase, segment,
    atom, position) equals the oracle's even/odd emulation; applied changes
    agree to 1e-9 relative.
  * FP32 policy: relative objective error <= 1e-6 and
    max |z - z_oracle| <= 1e-4 max |z_oracle| (both eps-solutions), and the
    returned Z passes the stop test max |Delta Z| < eps when the oracle
    recomputes beta from scratch.
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


def ctx_of(d, **cfg):
    cfg.setdefault("max_phases", 50_000)      # bound the host loop of a broken run
    return d.Context(**cfg)


def small(seed):
    return synth.workload(synth.SMALL, seed)


def f64(a):
    return np.asarray(a, dtype=np.float64)


# ------------------------------------------------------------- a1: S table

@pytest.mark.parametrize("K,P,W", [(5, 1, 32), (25, 7, 200), (3, 2, 5), (37, 3, 17)])
def test_s_table_matches_oracle(dicod, K, P, W):
    print(f"\ncase: S table K={K} P={P} W={W}", flush=True)
    _, D, _ = synth.generate(P, K, W, 4 * W, 0.01, 0.1, seed=K + W)
    with ctx_of(dicod) as c:
        c.set_dictionary(D)
        S_dev, n2 = c.s_table()
    S_o = oracle.s_table(f64(D))               # S_o[k, l] = S_{k,l}
    np.testing.assert_allclose(S_dev, S_o.transpose(1, 0, 2), rtol=0, atol=1e-13)
    np.testing.assert_allclose(n2, oracle.norms(f64(D)), rtol=0, atol=1e-14)


# ------------------------------------------------------------- a2: beta init

@pytest.mark.parametrize("K,P,W,T", [(5, 1, 32, 4096), (37, 3, 17, 1013), (25, 7, 200, 150_000),
                                     (2, 1, 1, 300), (4, 2, 9, 9)])
def test_beta_init_matches_oracle(dicod, K, P, W, T):
    print(f"\ncase: beta init K={K} P={P} W={W} T={T}", flush=True)
    X, D, _ = synth.generate(P, K, W, T, 0.01, 0.1, seed=T)
    with ctx_of(dicod) as c:
        c.set_dictionary(D)
        B = c.correlate(X)
    Bo = oracle.correlate(f64(D), f64(X))
    scale = max(1.0, float(np.abs(Bo).max()))
    np.testing.assert_allclose(B, Bo, rtol=0, atol=1e-12 * scale)


# ------------------------------------- a4-a9: FP64 trajectory = oracle even/odd

def _sorted_gpu_trace(tr):
    order = np.lexsort((tr["n_local"], tr["seg"], tr["phase"]))
    return tr[order]


def _sorted_oracle_trace(tr):
    order = np.lexsort((tr["n_local"], tr["seg"], tr["phase"]))
    return tr[order]


@pytest.mark.parametrize("M,cap,lds,C", [(4, 0, 1, 2), (4, 1, 1, 2), (4, 8, 1, 2), (1, 0, 1, 2),
                                         (63, 16, 1, 2), (4, 8, 0, 2), (63, 16, 0, 2),
                                         (127, 16, 1, 3), (127, 4, 0, 3), (90, 8, 1, 4),
                                         (5, 0, 1, 3)])
@pytest.mark.parametrize("seed", [0, 1])
def test_fp64_trajectory_matches_oracle(dicod, M, cap, lds, C, seed):
    """Both phase kernels (state in LDS, state in HBM) reproduce the oracle's
    coloured-phase sequence of updates (C = 2: even/odd); M = 1 is Algorithm 1
    (greedy CD)."""
    print(f"\ncase: FP64 trajectory small seed={seed} M={M} cap={cap} lds={lds} C={C}",
          flush=True)
    X, D, _ = small(seed)
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    Zo, so, tro = oracle.lgcd(f64(X), f64(D), lam, EPS, M, cap=cap, trace_cap=10**6, colors=C)
    with ctx_of(dicod, precision=dicod.DICOD_PREC_FP64, update_cap=cap,
                trace_capacity=10**6, state_in_lds=lds, colors=C) as c:
        Z, st = c.solve(X, lam, EPS, n_seg=M, D=D)
        tr = c.trace()
    assert st["state_in_hbm"] == (1 if (lds == 0 or M == 1) else 0)
    assert st["converged"] == 1 and so["converged"] == 1
    assert st["n_updates"] == so["n_updates"] == len(tr)
    assert st["n_phases"] == so["n_phases"]
    a, b = _sorted_gpu_trace(tr), _sorted_oracle_trace(tro)
    assert np.array_equal(a["phase"], b["phase"])
    assert np.array_equal(a["seg"], b["seg"])
    assert np.array_equal(a["k0"], b["k0"])
    assert np.array_equal(a["t0"], b["t0"])
    np.testing.assert_allclose(a["delta"], b["z_new"] - b["z_old"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Z, Zo, rtol=0, atol=1e-10)
    assert np.array_equal(Z != 0, Zo != 0)
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    assert abs(st["objective"] - Eo) <= 1e-10 * Eo


@pytest.mark.parametrize("M,cap,lds,C", [(4, 8, 1, 2), (63, 16, 0, 2), (127, 4, 1, 3),
                                         (1, 0, 1, 2)])
@pytest.mark.parametrize("seed", [0, 1])
def test_fp64_trajectory_matches_oracle_unequal_norms(dicod, M, cap, lds, C, seed):
    """The same sequence equality with atoms of norms spread over [0.3, 3], so the
    division by |D_k|^2 of eq. (pb_coord) acts: the GPU's g-form candidate
    (g - lambda sign beta) / |D_k|^2 against the oracle's Sh(beta, lambda) /
    |D_k|^2 - z, the Z it applies and the stop test."""
    print(f"\ncase: FP64 trajectory unequal norms seed={seed} M={M} cap={cap} lds={lds} "
          f"C={C}", flush=True)
    X, D, _ = small(seed)
    rng = np.random.default_rng(100 + seed)
    Dn = f64(D) / np.sqrt(np.sum(f64(D) ** 2, axis=(1, 2), keepdims=True))
    nrm = np.geomspace(0.3, 3.0, D.shape[0])[rng.permutation(D.shape[0])]
    D = (Dn * nrm[:, None, None]).astype(np.float32)
    n2 = oracle.norms(f64(D))
    assert n2.min() < 0.1 and n2.max() > 8.9
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    Zo, so, tro = oracle.lgcd(f64(X), f64(D), lam, EPS, M, cap=cap, trace_cap=10**6, colors=C)
    with ctx_of(dicod, precision=dicod.DICOD_PREC_FP64, update_cap=cap,
                trace_capacity=10**6, state_in_lds=lds, colors=C) as c:
        Z, st = c.solve(X, lam, EPS, n_seg=M, D=D)
        tr = c.trace()
    assert st["converged"] == 1 and so["converged"] == 1
    assert st["n_updates"] == so["n_updates"] == len(tr)
    assert st["n_phases"] == so["n_phases"]
    a, b = _sorted_gpu_trace(tr), _sorted_oracle_trace(tro)
    for f in ("phase", "seg", "k0", "t0"):
        assert np.array_equal(a[f], b[f]), f
    np.testing.assert_allclose(a["delta"], b["z_new"] - b["z_old"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(Z, Zo, rtol=0, atol=1e-10 * max(1.0, np.abs(Zo).max()))
    assert np.array_equal(Z != 0, Zo != 0)
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    assert abs(st["objective"] - Eo) <= 1e-10 * Eo


# ------------------------------------- MIXED: split-bf16 beta at Z = 0

@pytest.mark.parametrize("K,P,W,T", [(5, 1, 32, 4096), (37, 3, 17, 1013), (25, 7, 200, 150_000),
                                     (2, 1, 1, 300), (4, 2, 9, 9)])
def test_beta_init_split_bf16_error_bound(dicod, K, P, W, T):
    """bf16 rounding to nearest has unit roundoff u = 2^-8.  Split bf16 keeps
    hi = bf16(x) and lo = bf16(x - hi): |lo| <= u |x| and |x - hi - lo| <= u^2 |x|,
    so hi_d hi_x + hi_d lo_x + lo_d hi_x misses at most (3 u^2 + O(u^3)) |d x| of
    each product (lo_d lo_x and the two remainders), and fp32 accumulation of the
    P W terms adds at most P W 2^-24 of their absolute sum:
    |beta_mixed - beta| <= (3.1 * 2^-16 + P W 2^-24) sum |d| |x|."""
    print(f"\ncase: split-bf16 beta K={K} P={P} W={W} T={T}", flush=True)
    X, D, _ = synth.generate(P, K, W, T, 0.01, 0.1, seed=T + 1)
    with ctx_of(dicod) as c:
        c.set_dictionary(D)
        B = c.correlate(X, precision=dicod.DICOD_PREC_MIXED)
    Bo = oracle.correlate(f64(D), f64(X))
    A = oracle.correlate(np.abs(f64(D)), np.abs(f64(X)))
    bound = (3.1 * 2.0 ** -16 + P * W * 2.0 ** -24) * A + 1e-30
    err = np.abs(B - Bo)
    print(f"max error / bound {np.max(err / bound):.3f}, max rel to sum|dx| "
          f"{np.max(err / (A + 1e-30)):.3g}", flush=True)
    assert np.all(err <= bound)


def test_paper_shaped_mixed_matches_oracle(dicod, paper_problem):
    print("\ncase: MIXED paper-shaped P=7 K=25 W=200 T=150000", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod, precision=dicod.DICOD_PREC_MIXED) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    print(f"gpu: {st['n_updates']} updates, rounds {st['round_updates']}, "
          f"init {st['t_init_ms']:.3f} cd {st['t_cd_ms']:.3f} verify {st['t_verify_ms']:.3f} ms",
          flush=True)
    assert abs(st["lambda"] - lam) <= 1e-12 * lam   # exact lambda_max refinement
    _check_solution(X, D, lam, Z, st, Zo)


def test_mixed_lambda_max_exact_when_bf16_ranking_is_wrong(dicod):
    """X = 1e6 u + v with u in the null space of X -> D^T X (dimension T - L =
    W - 1): the correlation of X is about that of v, but the split-bf16
    rounding error scales with sum |d| |x| ~ 1e6, far above the gaps between
    the largest entries, so a refinement window fixed relative to the
    split-bf16 maximum misses the maximiser.  lambda_max must still equal the
    double-precision maximum of D^T X (its definition, eq. (2))."""
    rng = np.random.default_rng(21)
    K, P, W, T = 1, 1, 16, 64
    D = rng.standard_normal((K, P, W))
    D /= np.linalg.norm(D)
    D = D.astype(np.float32)
    L = T - W + 1
    C = np.zeros((L, T))
    for t in range(L):
        C[t, t:t + W] = f64(D[0, 0])
    _, sv, Vt = np.linalg.svd(C)
    u = Vt[-1]                                   # C u = 0
    assert sv[-1] < 1e-12 * sv[0] or np.abs(C @ u).max() < 1e-12
    X = (1e6 * u + rng.standard_normal(T)).astype(np.float32)[None, :]
    B = oracle.correlate(f64(D), f64(X))
    lmax = float(np.max(np.abs(B)))
    scale = float(np.sum(np.abs(f64(X))) * np.abs(f64(D)).max())
    with ctx_of(dicod, precision=dicod.DICOD_PREC_MIXED) as c:
        c.set_dictionary(D)
        Bm = c.correlate(X, precision=dicod.DICOD_PREC_MIXED)
        _, st = c.solve(X, -0.1, EPS, n_seg=1)
    print(f"lambda_max {lmax:.6f}; split-bf16 argmax {np.argmax(np.abs(Bm))} vs exact "
          f"{np.argmax(np.abs(B))}; max error {np.abs(Bm - B).max():.3g}", flush=True)
    gap = np.sort(np.abs(B).ravel())[-1] - np.sort(np.abs(B).ravel())[-2]
    assert np.abs(Bm - B).max() > max(1e-3 * lmax, gap)     # split-bf16 cannot rank
    assert abs(st["lambda_max"] - lmax) <= 1e-13 * scale


# ------------------------------------------------ FP32 policy: eps-solutions

def _check_solution(X, D, lam, Z, st, Zo):
    Eo = oracle.objective(f64(X), f64(D), Zo, lam)
    E = oracle.objective(f64(X), f64(D), Z, lam)
    assert abs(E - Eo) <= 1e-6 * Eo, (E, Eo)
    assert abs(st["objective"] - E) <= 1e-9 * E
    assert np.max(np.abs(Z - Zo)) <= 1e-4 * np.max(np.abs(Zo))
    assert st["converged"] == 1 and st["max_dz"] < EPS
    mdz, _, _ = oracle.max_dz(f64(X), f64(D), Z, lam)
    assert mdz < EPS * (1 + 1e-6), mdz


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("M", [4, 0])
def test_fp32_small_matches_oracle(dicod, seed, M):
    print(f"\ncase: FP32 small seed={seed} M={M}", flush=True)
    X, D, _ = small(seed)
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    Zo, so, _ = oracle.lgcd(f64(X), f64(D), lam, EPS, 4, cap=16)
    with ctx_of(dicod) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=M, D=D)   # relative lambda
    assert abs(st["lambda"] - lam) <= 1e-12 * lam
    _check_solution(X, D, lam, Z, st, Zo)


def test_paper_shaped_fp32_matches_oracle(dicod, paper_problem):
    print("\ncase: FP32 paper-shaped P=7 K=25 W=200 T=150000 (auto segments)", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    print(f"gpu: {st['n_updates']} updates, {st['n_phases']} phases, M={st['n_seg']}, "
          f"refresh={st['n_refresh']}, cd={st['t_cd_ms']:.2f} ms", flush=True)
    assert st["n_seg"] == 752   # floor(L / (W - 1)) for 3 colours
    _check_solution(X, D, lam, Z, st, Zo)
    # phases queued past a round's convergence apply nothing and are not
    # counted: n_phases is the rounds' phases plus at most C - 1 alignment
    # phases before each resumed round
    rp = [p for p in st["round_phases"] if p > 0]
    assert sum(rp) <= st["n_phases"] <= sum(rp) + 2 * (len(rp) - 1)
    assert st["n_phase_launches"] >= sum(rp)


@pytest.fixture(scope="module")
def paper_problem():
    X, D, _ = synth.workload(synth.PAPER, 0)
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    Zo, so, _ = oracle.lgcd(f64(X), f64(D), lam, EPS, 374, cap=16)
    return X, D, lam, Zo


@pytest.mark.parametrize("M", [8, 32, 128, 256])
def test_paper_shaped_segment_sweep(dicod, paper_problem, M):
    """Few long segments run with the state in HBM; every segment count gives
    an eps-solution of the same problem."""
    print(f"\ncase: paper-shaped FP32 M={M}", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=M, D=D)
    print(f"gpu: {st['n_updates']} updates, {st['n_phases']} phases, hbm={st['state_in_hbm']}, "
          f"cd={st['t_cd_ms']:.2f} ms", flush=True)
    assert st["n_seg"] == M
    _check_solution(X, D, lam, Z, st, Zo)


@pytest.mark.parametrize("lds", [1, 0])
def test_paper_shaped_fp64(dicod, paper_problem, lds):
    """Double state of the paper-shaped segments: on chip (own positions in
    LDS, halo changes applied in HBM) or, forced, entirely in HBM."""
    print(f"\ncase: paper-shaped FP64 state_in_lds={lds}", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod, precision=dicod.DICOD_PREC_FP64, state_in_lds=lds) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    assert st["state_in_hbm"] == 1 - lds and st["n_refresh"] == 0
    _check_solution(X, D, lam, Z, st, Zo)


@pytest.mark.parametrize("polish", [0, 1, 2])
def test_paper_shaped_fp32_polish_policies(dicod, paper_problem, polish):
    print(f"\ncase: paper-shaped FP32 fp64_polish_after={polish}", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod, fp64_polish_after=polish) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    print(f"gpu: rounds {st['round_updates']} / {st['round_phases']}, refresh={st['n_refresh']}, "
          f"polished={st['polished_fp64']}, cd={st['t_cd_ms']:.2f} verify={st['t_verify_ms']:.2f}",
          flush=True)
    _check_solution(X, D, lam, Z, st, Zo)


def test_state_check_agrees_with_recompute(dicod, paper_problem):
    """The final stop test on the maintained double state and the one that
    recomputes g from Z in double see the same iterate and agree."""
    X, D, lam, Zo = paper_problem
    out = []
    for scratch in (0, 1):
        with ctx_of(dicod, verify_from_scratch=scratch) as c:
            out.append(c.solve(X, -0.1, EPS, n_seg=0, D=D))
    (Z0, s0), (Z1, s1) = out
    assert np.array_equal(Z0, Z1)
    # the residual energy comes from g (|X|^2 - <beta0 + g, Z>): the two g
    # agree to rounding, and so do the objectives
    assert abs(s0["objective"] - s1["objective"]) <= 1e-12 * s1["objective"]
    assert abs(s0["max_dz"] - s1["max_dz"]) <= 1e-12
    assert abs(s0["kkt_on"] - s1["kkt_on"]) <= 1e-12 and abs(s0["kkt_off"] - s1["kkt_off"]) <= 1e-12
    _check_solution(X, D, lam, Z0, s0, Zo)


# ------------------------------------------------------------- edge cases

def test_lambda_at_lambda_max_gives_zero(dicod):
    X, D, _ = small(4)
    with ctx_of(dicod) as c:
        Z, st = c.solve(X, -1.0, EPS, n_seg=4, D=D)
    assert st["n_updates"] == 0 and not Z.any() and st["converged"] == 1
    assert st["objective"] == pytest.approx(0.5 * float(np.sum(f64(X) ** 2)), rel=1e-12)


@pytest.mark.parametrize("prec", ["FP64", "FP32", "MIXED"])
@pytest.mark.parametrize("K,P,W,T,M", [
    (1, 1, 8, 8, 1),          # L = 1
    (3, 2, 5, 200, 1),        # single segment, generic K
    (3, 4, 5, 333, 7),        # ragged segments (L = 329 = 7 * 47)
    (25, 7, 20, 5003, 13),    # K = 25 kernel, ragged tail
    (40, 2, 6, 900, 5),       # K > 32: two atom blocks in the check kernels
    (64, 16, 16, 2000, 8),    # largest K of the LDS-state kernel, largest P
    (66, 3, 8, 200, 1),       # K > 64: state in HBM for every precision
    (4, 2, 700, 6000, 3),     # wide atoms: several tau passes, windows of 1399 positions
    (3, 2, 1, 300, 5),        # W = 1: no coupling between positions
])
def test_shapes_match_oracle(dicod, prec, K, P, W, T, M):
    print(f"\ncase: shape {prec} K={K} P={P} W={W} T={T} M={M}", flush=True)
    X, D, _ = synth.generate(P, K, W, T, 0.05, 0.1, seed=7 * T + K)
    lam = 0.15 * oracle.lambda_max(f64(X), f64(D))
    Zo, so, _ = oracle.lgcd(f64(X), f64(D), lam, 1e-10, M)
    p = getattr(dicod, f"DICOD_PREC_{prec}")
    with ctx_of(dicod, precision=p) as c:
        Z, st = c.solve(X, lam, EPS, n_seg=M, D=D)
    _check_solution(X, D, lam, Z, st, Zo)


@pytest.mark.parametrize("prec", ["FP64", "FP32", "MIXED"])
def test_zero_signal_gives_zero(dicod, prec):
    # X = 0: lambda_max = 0, Z = 0 is the solution for every lambda >= 0 and
    # the cost is 0; a relative lambda becomes 0, an absolute one stays.
    _, D, _ = small(5)
    X = np.zeros((D.shape[1], 3000), dtype=np.float32)
    p = getattr(dicod, f"DICOD_PREC_{prec}")
    for lam in (-0.1, 0.25):
        print(f"\ncase: zero signal {prec} lam={lam}", flush=True)
        with ctx_of(dicod, precision=p) as c:
            Z, st = c.solve(X, lam, EPS, n_seg=6, D=D)
        assert not Z.any() and st["n_updates"] == 0 and st["converged"] == 1
        assert st["objective"] == 0.0 and st["lambda_max"] == 0.0


@pytest.mark.parametrize("bad", ["lam0", "lamnan", "eps0", "short_segments", "T_lt_W",
                                 "nan_x", "zero_atom", "n_seg_gt_L"])
def test_invalid_arguments_rejected(dicod, bad):
    X, D, _ = small(0)
    lam, eps, M = -0.1, EPS, 4
    if bad == "lam0":
        lam = 0.0
    elif bad == "lamnan":
        lam = float("nan")
    elif bad == "eps0":
        eps = 0.0
    elif bad == "short_segments":
        M = 200                      # 4065 / 200 < W = 32
    elif bad == "T_lt_W":
        X = X[:, :16]
    elif bad == "nan_x":
        X = X.copy()
        X[0, 5] = np.nan
    elif bad == "zero_atom":
        D = D.copy()
        D[2] = 0
    elif bad == "n_seg_gt_L":
        X = X[:, :40]
        M = 20
    with ctx_of(dicod) as c:
        with pytest.raises(dicod.DicodError) as e:
            c.solve(X, lam, eps, n_seg=M, D=D)
        assert e.value.code == dicod.DICOD_EINVAL
        assert dicod.dicod_last_error(c.h)


# ------------------------------------------------- device API and batching

def test_device_api_equals_host_api(dicod):
    import torch
    X, D, _ = small(5)
    with ctx_of(dicod) as c:
        Zh, sh = c.solve(X, -0.1, EPS, n_seg=4, D=D)
        Xd = torch.from_numpy(X).cuda()
        Zd, sd, _ = c.solve_device(Xd, -0.1, EPS, n_seg=4)
        torch.cuda.synchronize()
    assert np.array_equal(Zd.cpu().numpy(), Zh)
    assert sd["n_updates"] == sh["n_updates"]


@pytest.mark.parametrize("polish", [1, 0, 2])
def test_batch_equals_solo_bitwise(dicod, polish):
    """A batched solve equals the solo solves element by element for every
    polish policy (a signal whose stop test held is frozen while the others
    continue), and every signal is an eps-solution of the oracle's problem."""
    import torch
    print(f"\ncase: batch vs solo polish={polish}", flush=True)
    P, K, W = 7, 25, 64
    lens = [12_000, 3_001, 20_500, 9_999]
    _, D, _ = synth.generate(P, K, W, 4 * W, 0.005, 0.1, seed=11)
    sigs = [synth.generate(P, K, W, T, 0.005, 0.1, seed=100 + i, D=D)[0]
            for i, T in enumerate(lens)]
    Ls = [T - W + 1 for T in lens]
    x_off = np.cumsum([0] + [P * T for T in lens[:-1]])
    z_off = np.cumsum([0] + [K * L for L in Ls[:-1]])
    with ctx_of(dicod, fp64_polish_after=polish) as c:
        c.set_dictionary(D)
        solo = []
        for X in sigs:
            Z, st, _ = c.solve_device(torch.from_numpy(X).cuda(), -0.1, EPS)
            solo.append((Z.cpu().numpy(), st))
        Xall = torch.from_numpy(np.concatenate([x.reshape(-1) for x in sigs])).cuda()
        Zall = torch.zeros(int(sum(K * L for L in Ls)), dtype=torch.float64, device="cuda")
        sts = c.solve_batch_device(Xall, lens, x_off, [-0.1] * len(lens), EPS, None, Zall,
                                   z_off)
        torch.cuda.synchronize()
        Zall = Zall.cpu().numpy()
    for i, (Zs, st) in enumerate(solo):
        Zb = Zall[z_off[i]:z_off[i] + K * Ls[i]].reshape(K, Ls[i])
        assert np.array_equal(Zb, Zs), f"signal {i} differs between batch and solo"
        assert sts[i]["n_updates"] == st["n_updates"]
        assert sts[i]["converged"] == 1
        X = sigs[i]
        lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
        assert abs(sts[i]["lambda"] - lam) <= 1e-12 * lam
        Zo, _, _ = oracle.lgcd(f64(X), f64(D), lam, 1e-10, max(1, Ls[i] // 400))
        _check_solution(X, D, lam, Zb, sts[i], Zo)


# ------------------------------------------- long signal: sampled oracle checks

@pytest.mark.parametrize("policy", ["fp32", "mixed_float_only"])
def test_long_signal_sampled_against_oracle(dicod, policy):
    """T = 5,000,000 (P=7, K=25, W=200): too long for an oracle solve, so the
    oracle recomputes beta from its definition at sampled coordinates (random
    non-zeros of Z and random coordinates) and the objective of the returned
    Z; every sampled |Delta Z| must be below eps (the stop test of Sec. 2.1)
    and the objective must agree with the library's double-precision value.
    Policies: FP32 (double beta, a double finish round after a failed check),
    and the long workload's own: split-bf16 correlations, float descent only
    (fp64_polish_after = 0), segments of at most 256 positions from a tuning
    entry."""
    import torch
    w = synth.LONG
    print(f"\ncase: long signal T={w.T} policy={policy}", flush=True)
    D = synth.dictionary(np.random.Generator(np.random.PCG64(31)), w.K, w.P, w.W).astype(np.float32)
    X = synth.generate_fast(w.P, w.K, w.W, w.T, w.rho, w.sigma_noise, 32, D)
    print("inputs ready", flush=True)
    cfg = {} if policy == "fp32" else dict(precision=dicod.DICOD_PREC_MIXED,
                                           fp64_polish_after=0, autotune=1)
    with ctx_of(dicod, **cfg) as c:
        c.set_dictionary(D)
        if policy != "fp32":
            c.set_tuning(dict(K=w.K, P=w.P, W=w.W, bucket=22, colors=3, seg_len=256,
                              update_cap=28))
        Xd = torch.from_numpy(X).cuda()
        Zd, st, _ = c.solve_device(Xd, -w.lam_rel, EPS)
        Z = Zd.cpu().numpy()
    print(f"gpu: {st['n_updates']} updates, {st['n_phases']} phases, M={st['n_seg']}, "
          f"time {st['t_total_ms']:.1f} ms, max_dz {st['max_dz']:.3g}, rounds "
          f"{st['round_state']}", flush=True)
    assert st["converged"] == 1 and st["max_dz"] < EPS
    if policy != "fp32":
        assert st["tuned"] == 1 and st["polished_fp64"] == 0
        assert all(s & 1 == 0 for s in st["round_state"])   # no double descent round
    assert st["lambda"] == pytest.approx(w.lam_rel * st["lambda_max"], rel=1e-15)
    K, L = Z.shape
    rng = np.random.default_rng(5)
    nzk, nzt = np.nonzero(Z)
    pick = rng.choice(nzk.size, size=min(3000, nzk.size), replace=False)
    k = np.concatenate([nzk[pick], rng.integers(0, K, 3000)])
    t = np.concatenate([nzt[pick], rng.integers(0, L, 3000)])
    B = oracle.beta_at(f64(X), f64(D), Z, k, t)
    n2 = oracle.norms(f64(D))
    lam = st["lambda"]
    zp = np.sign(B) * np.maximum(np.abs(B) - lam, 0.0) / n2[k]
    dz = np.abs(zp - Z[k, t])
    print(f"sampled max |Delta Z| {dz.max():.3g} over {dz.size} coordinates", flush=True)
    assert dz.max() < EPS
    # every coordinate within W - 1 of 200 segment edges (where the halo
    # records of boundary updates act; segments b_m = floor(m L / M)): beta
    # from its definition on a local problem covering Z on [e - 2W + 2,
    # e + 2W - 2), which is exact on [e - W + 1, e + W - 1)
    W = w.W
    M = st["n_seg"]
    edges = (np.sort(rng.choice(np.arange(1, M), size=200, replace=False)).astype(np.int64)
             * L) // M
    worst = 0.0
    n_chk = 0
    for e in edges:
        s0, s1 = e - 2 * W + 2, e + 2 * W - 2
        if s0 < 0 or s1 > L:
            continue
        Bl = oracle.beta(f64(X[:, s0:s1 + W - 1]), f64(D), Z[:, s0:s1])
        Bl = Bl[:, W - 1:3 * W - 3]
        Zl = Z[:, e - W + 1:e + W - 1]
        zp = np.sign(Bl) * np.maximum(np.abs(Bl) - lam, 0.0) / n2[:, None]
        worst = max(worst, float(np.abs(zp - Zl).max()))
        n_chk += Zl.size
    print(f"edge bands: max |Delta Z| {worst:.3g} over {n_chk} coordinates", flush=True)
    assert n_chk > 150 * K * (2 * W - 2) and worst < EPS
    obj = oracle.objective(f64(X), f64(D), Z, lam)
    assert abs(obj - st["objective"]) <= 1e-10 * abs(obj)


# ------------------------------- f1: Algorithm 2 in lockstep (DICOD schedule)

def interference_from_trace(phase, seg, k0, t0, delta, S, W):
    """Concurrent updates of adjacent segments in one phase: pair count, pairs
    with |t0 - t1| < W (interfering, Sec. 3) and their Prop. A.2 terms."""
    by = {}
    for p, m, k, t, d in zip(phase, seg, k0, t0, delta):
        by.setdefault((int(p), int(m)), []).append((int(k), int(t), float(d)))
    n_adj = n_int = 0
    acc = 0.0
    for (p, m), us in by.items():
        vs = by.get((p, m + 1))
        if not vs:
            continue
        for ku, tu, du in us:
            for kv, tv, dv in vs:
                n_adj += 1
                dt = tu - tv
                if -W < dt < W:
                    n_int += 1
                    acc += S[ku, kv, dt + W - 1] * du * dv
    return n_adj, n_int, acc


DICOD_CASES = [  # (workload, M, cap): segments >= W
    ("small", 4, 1), ("small", 16, 1), ("small", 64, 1), ("small", 64, 4),
    ("k25", 13, 1), ("k25", 100, 2),
]


def _dicod_problem(name, seed):
    if name == "small":
        return small(seed)
    return synth.generate(7, 25, 20, 5003, 0.02, 0.1, seed=40 + seed)


@pytest.mark.parametrize("name,M,cap", DICOD_CASES)
@pytest.mark.parametrize("seed", [0, 1])
def test_dicod_schedule_fp64_trajectory_matches_oracle(dicod, name, M, cap, seed):
    print(f"\ncase: DICOD schedule FP64 {name} M={M} cap={cap} seed={seed}", flush=True)
    X, D, _ = _dicod_problem(name, seed)
    W = D.shape[2]
    lam = 0.1 * oracle.lambda_max(f64(X), f64(D))
    n = 200_000
    Zo, so, tro = oracle.lgcd(f64(X), f64(D), lam, EPS, M, schedule=oracle.SCHED_DICOD,
                              cap=cap, trace_cap=n)
    assert so["converged"] == 1
    with ctx_of(dicod, precision=dicod.DICOD_PREC_FP64, schedule=dicod.DICOD_SCHED_DICOD,
                update_cap=cap, trace_capacity=n) as c:
        Z, st = c.solve(X, lam, EPS, n_seg=M, D=D)
        tr = _sorted_gpu_trace(c.trace())
    print(f"oracle: {so['n_updates']} updates, {so['n_phases']} phases, {so['n_interf']} "
          f"interfering of {so['n_adjacent']} adjacent pairs; gpu: {st['n_updates']} updates",
          flush=True)
    assert st["n_refresh"] == 0 and st["converged"] == 1
    assert len(tr) == len(tro) == so["n_updates"]
    for f in ("phase", "seg", "k0", "t0", "n_local"):
        np.testing.assert_array_equal(tr[f], tro[f], err_msg=f)
    d_o = tro["z_new"] - tro["z_old"]
    np.testing.assert_allclose(tr["delta"], d_o, rtol=1e-9, atol=1e-12 * np.abs(d_o).max())
    S = oracle.s_table(f64(D))
    n_adj, n_int, acc = interference_from_trace(tr["phase"], tr["seg"], tr["k0"], tr["t0"],
                                                tr["delta"], S, W)
    assert (n_adj, n_int) == (so["n_adjacent"], so["n_interf"])
    assert abs(acc - so["interf_sum"]) <= 1e-9 * max(1.0, abs(so["interf_sum"]))
    np.testing.assert_allclose(Z, Zo, rtol=0, atol=1e-9 * np.abs(Zo).max())


def test_dicod_schedule_fp32_paper_shaped(dicod, paper_problem):
    print("\ncase: DICOD schedule FP32 paper-shaped", flush=True)
    X, D, lam, Zo = paper_problem
    with ctx_of(dicod, schedule=dicod.DICOD_SCHED_DICOD, update_cap=1) as c:
        Z, st = c.solve(X, -0.1, EPS, n_seg=0, D=D)
    print(f"gpu: {st['n_updates']} updates, {st['n_phases']} phases, M={st['n_seg']}, "
          f"rounds {st['round_updates']}, cd {st['t_cd_ms']:.2f} ms", flush=True)
    assert st["n_seg"] == 752   # floor(L / (W - 1)) for 3 colours
    _check_solution(X, D, lam, Z, st, Zo)


@pytest.mark.parametrize("bad", ["cap0", "short"])
def test_dicod_schedule_rejects(dicod, bad):
    X, D, _ = small(0)
    if bad == "cap0":
        with pytest.raises(dicod.DicodError) as ei:
            ctx_of(dicod, schedule=dicod.DICOD_SCHED_DICOD, update_cap=0)
        assert ei.value.code == dicod.DICOD_EINVAL
        return
    with ctx_of(dicod, schedule=dicod.DICOD_SCHED_DICOD, update_cap=1) as c:
        with pytest.raises(dicod.DicodError) as ei:
            c.solve(X, -0.1, EPS, n_seg=200, D=D)   # segments of 20 < W = 32
        assert ei.value.code == dicod.DICOD_EINVAL
