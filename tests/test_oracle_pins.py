"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: each compares it with a
library routine, a brute-force evaluation of a definition, a closed form, a
hand-derived example or an invariant the paper proves.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_problem(seed, P=2, K=3, W=5, T=40, rho=0.08, noise=0.1):
    X, D, Zt = synth.generate(P, K, W, T, rho, noise, seed)
    return X.astype(np.float64), D.astype(np.float64), Zt


# ---------------------------------------------------------------- primitives

def test_soft_threshold_hand_values():
    # Sh(u, lambda) = sign(u) max(|u| - lambda, 0)  (Sec. 2.1)
    assert oracle.soft_threshold(3.0, 1.0) == 2.0
    assert oracle.soft_threshold(-3.0, 1.0) == -2.0
    assert oracle.soft_threshold(-0.5, 1.0) == 0.0
    assert oracle.soft_threshold(1.0, 1.0) == 0.0
    assert oracle.soft_threshold(0.25, 0.0) == 0.25


def test_s_table_matches_numpy_correlate():
    # S_{k,l}[d] = sum_tau <D_k[tau], D_l[tau+d]> via numpy.correlate ('full').
    _, D, _ = tiny_problem(1, P=3, K=4, W=7)
    K, P, W = D.shape
    S = oracle.s_table(D)
    for k in range(K):
        for l in range(K):
            ref = sum(np.correlate(D[l, p], D[k, p], mode="full") for p in range(P))
            np.testing.assert_allclose(S[k, l], ref, rtol=0, atol=1e-14)
    # symmetry S_{k,l}[d] = S_{l,k}[-d] and S_{k,k}[0] = |D_k|^2
    np.testing.assert_allclose(S, np.transpose(S, (1, 0, 2))[:, :, ::-1], atol=1e-15)
    np.testing.assert_allclose(np.diagonal(S[:, :, W - 1]), oracle.norms(D), atol=1e-15)


def test_correlate_matches_numpy():
    X, D, _ = tiny_problem(2, P=3, K=4, W=6, T=50)
    K, P, W = D.shape
    B = oracle.correlate(D, X)
    for k in range(K):
        ref = sum(np.correlate(X[p], D[k, p], mode="valid") for p in range(P))
        np.testing.assert_allclose(B[k], ref, rtol=0, atol=1e-13)


def test_reconstruct_matches_numpy_convolve():
    X, D, Zt = tiny_problem(3, P=2, K=3, W=5, T=30, rho=0.3)
    K, P, W = D.shape
    T = X.shape[1]
    R = oracle.reconstruct(D, Zt, T)
    ref = np.zeros((P, T))
    for k in range(K):
        for p in range(P):
            ref[p] += np.convolve(Zt[k], D[k, p], mode="full")
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-12)


def _beta_by_definition(X, D, Z):
    """beta_k[t]: correlate D_k with X - sum_{k'} Z_{k'} * D_{k'} where Z_k[t] alone
    is replaced by 0 (the replacement operator Phi_t of Sec. 2)."""
    K, P, W = D.shape
    T = X.shape[1]
    L = T - W + 1
    out = np.zeros((K, L))
    for k in range(K):
        for t in range(L):
            Zm = Z.copy()
            Zm[k, t] = 0.0
            R = X.copy()
            for kk in range(K):
                for p in range(P):
                    R[p] -= np.convolve(Zm[kk], D[kk, p], mode="full")
            out[k, t] = sum(np.dot(D[k, p], R[p, t:t + W]) for p in range(P))
    return out


def test_beta_matches_definition_with_replacement_operator():
    X, D, Zt = tiny_problem(4, P=2, K=2, W=4, T=20, rho=0.3)
    np.testing.assert_allclose(oracle.beta(X, D, Zt), _beta_by_definition(X, D, Zt),
                               rtol=0, atol=1e-12)


def test_beta_at_matches_definition():
    # sampled beta (one coordinate at a time, from the window's residual)
    X, D, Zt = tiny_problem(6, P=2, K=3, W=5, T=30, rho=0.3)
    K, L = Zt.shape
    kk, tt = np.meshgrid(np.arange(K), np.arange(L), indexing="ij")
    B = oracle.beta_at(X, D, Zt, kk.ravel(), tt.ravel()).reshape(K, L)
    np.testing.assert_allclose(B, _beta_by_definition(X, D, Zt), rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        oracle.beta_at(X, D, Zt, [0], [L])


# ------------------------------------------------------------ solver checks

def _greedy_brute_force(X, D, lam, eps, n_steps):
    """Algorithm 1 with beta recomputed from its definition at every step."""
    K, P, W = D.shape
    L = X.shape[1] - W + 1
    n2 = np.sum(D * D, axis=(1, 2))
    Z = np.zeros((K, L))
    steps = []
    for _ in range(n_steps):
        B = _beta_by_definition(X, D, Z)
        Zp = np.sign(B) * np.maximum(np.abs(B) - lam, 0.0) / n2[:, None]
        dz = np.abs(Zp - Z)
        # argmax with ties to the smallest t, then the smallest k
        flat = np.argmax(dz.T.reshape(-1))
        t0, k0 = divmod(int(flat), K)
        if dz[k0, t0] < eps:
            break
        steps.append((k0, t0, Zp[k0, t0]))
        Z[k0, t0] = Zp[k0, t0]
    return Z, steps


@pytest.mark.parametrize("seed", [0, 5])
def test_single_segment_is_greedy_cd(seed):
    # M = 1: the locally greedy rule is the greedy rule of Algorithm 1; the
    # incremental beta of eq. (3) must reproduce the from-scratch trajectory.
    X, D, _ = tiny_problem(seed, P=2, K=2, W=4, T=24, rho=0.15)
    lam = 0.1 * oracle.lambda_max(X, D)
    n = 25
    Zb, steps = _greedy_brute_force(X, D, lam, 1e-9, n)
    for sched in (oracle.SCHED_EVENODD, oracle.SCHED_SEQUENCE):
        Z, st, tr = oracle.lgcd(X, D, lam, 1e-9, 1, schedule=sched,
                                seq=[0] if sched == oracle.SCHED_SEQUENCE else None,
                                max_steps=len(steps), trace_cap=n)
        assert len(tr) == len(steps)
        for rec, (k0, t0, zn) in zip(tr, steps):
            assert (rec["k0"], rec["t0"]) == (k0, t0)
            assert abs(rec["z_new"] - zn) <= 1e-10 * max(1.0, abs(zn))
        np.testing.assert_allclose(Z, Zb, atol=1e-10)


def test_prop_a1_cost_change_matches_objective():
    # Prop. A.1: per-update decrease equals E(Z) - E(Z') computed directly.
    X, D, _ = tiny_problem(6, P=2, K=3, W=5, T=60)
    lam = 0.1 * oracle.lambda_max(X, D)
    Zprev = np.zeros((3, 56))
    Eprev = oracle.objective(X, D, Zprev, lam)
    _, _, tr = oracle.lgcd(X, D, lam, 1e-8, 3, trace_cap=10)
    for j in range(1, 8):
        Z, _, _ = oracle.lgcd(X, D, lam, 1e-8, 3, max_steps=j)
        E = oracle.objective(X, D, Z, lam)
        assert abs((Eprev - E) - tr[j - 1]["dE"]) <= 1e-10 * max(1.0, abs(Eprev))
        Eprev = E


def test_monotone_decrease_and_lemma_a1_bound():
    # Convergence proof of Theorem 1: each sequential update decreases E;
    # Lemma A.1: the decrease is at least |D_k|^2 delta^2 / 2.
    X, D, _ = synth.workload(synth.SMALL, 2)
    lam = 0.1 * oracle.lambda_max(X, D)
    Z, st, tr = oracle.lgcd(X, D, lam, 1e-6, 4, cap=8, trace_cap=10**5)
    assert st["converged"] == 1
    n2 = oracle.norms(D)
    delta = tr["z_new"] - tr["z_old"]
    assert np.all(tr["dE"] > 0)
    assert np.all(tr["dE"] - 0.5 * n2[tr["k0"]] * delta ** 2 >= -1e-9 * np.maximum(1, tr["dE"]))
    E0 = oracle.objective(X, D, np.zeros_like(Z), lam)
    E1 = oracle.objective(X, D, Z, lam)
    assert abs((E0 - E1) - st["dE_sum"]) <= 1e-9 * E0


def test_lambda_at_or_above_lambda_max_gives_zero():
    X, D, _ = tiny_problem(7)
    lmax = oracle.lambda_max(X, D)
    Z, st, _ = oracle.lgcd(X, D, lmax * (1 + 1e-12), 1e-8, 2)
    assert st["n_updates"] == 0 and st["converged"] == 1
    assert not Z.any()
    Z, st, _ = oracle.lgcd(X, D, lmax * 0.99, 1e-8, 2)
    assert st["n_updates"] >= 1


def test_orthonormal_atoms_of_length_one_closed_form():
    # W = 1 and orthonormal atoms (P = K): the problem separates over t and
    # k and z_k[t] = Sh(<D_k, X[t]>, lambda).
    rng = np.random.default_rng(0)
    P = K = 4
    Q, _ = np.linalg.qr(rng.standard_normal((P, P)))
    D = Q.T[:, :, None].copy()           # D_k[p, 0] = Q[p, k]
    X = 3.0 * rng.standard_normal((P, 30))
    lam = 1.5
    Z, st, _ = oracle.lgcd(X, D, lam, 1e-12, 1)
    ref = Q.T @ X
    ref = np.sign(ref) * np.maximum(np.abs(ref) - lam, 0.0)
    np.testing.assert_allclose(Z, ref, atol=1e-12)
    assert st["n_updates"] == np.count_nonzero(ref)


def test_single_coordinate_closed_form():
    # T = W (L = 1), K = 1: z = Sh(<D, X>, lambda) / |D|^2 (eq. (pb_coord)).
    rng = np.random.default_rng(1)
    D = rng.standard_normal((1, 3, 6))
    X = rng.standard_normal((3, 6)) * 4
    lam = 0.7
    Z, _, _ = oracle.lgcd(X, D, lam, 1e-14, 1)
    u = float(np.sum(D[0] * X))
    ref = np.sign(u) * max(abs(u) - lam, 0.0) / float(np.sum(D * D))
    assert abs(Z[0, 0] - ref) <= 1e-14


def _read_golden():
    rows = []
    with open(os.path.join(GOLDEN, "two_coordinate_lasso.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, x, z, g = [s.split() for s in line.split("|")]
            rows.append((name[0], [Fraction(v) for v in x], [Fraction(v) for v in z],
                         [Fraction(v) for v in g]))
    return rows


@pytest.mark.parametrize("row", _read_golden(), ids=lambda r: r[0])
def test_golden_two_coordinate_lasso(row):
    _, x, z, _ = row
    D = np.array([[[0.6, 0.8]]])
    X = np.array([[float(v) for v in x]])
    for M, sched in ((1, oracle.SCHED_EVENODD), (2, oracle.SCHED_SEQUENCE)):
        Z, st, _ = oracle.lgcd(X, D, 0.5, 1e-14, M, schedule=sched,
                               seq=[0, 1] if sched == oracle.SCHED_SEQUENCE else None)
        assert st["converged"] == 1
        np.testing.assert_allclose(Z[0], [float(v) for v in z], atol=1e-12)


def _toeplitz_design(D, T):
    """Explicit Lasso design A in R^{PT x KL}: column (k, t) is D_k placed at t."""
    K, P, W = D.shape
    L = T - W + 1
    A = np.zeros((P * T, K * L))
    for k in range(K):
        for t in range(L):
            col = np.zeros((P, T))
            col[:, t:t + W] = D[k]
            A[:, k * L + t] = col.reshape(-1)
    return A


def _fista(A, x, lam, n_iter=20000, tol=1e-14):
    Lip = np.linalg.norm(A, 2) ** 2
    z = np.zeros(A.shape[1])
    y = z.copy()
    s = 1.0
    for _ in range(n_iter):
        u = y - A.T @ (A @ y - x) / Lip
        zn = np.sign(u) * np.maximum(np.abs(u) - lam / Lip, 0.0)
        sn = (1 + np.sqrt(1 + 4 * s * s)) / 2
        y = zn + (s - 1) / sn * (zn - z)
        if np.max(np.abs(zn - z)) < tol:
            z = zn
            break
        z, s = zn, sn
    return z


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_brute_force_explicit_toeplitz_lasso(seed):
    # Problem (2) is a Lasso with a banded Toeplitz design (Sec. 2.1); solve it
    # independently with FISTA on the explicit matrix.
    X, D, _ = tiny_problem(seed, P=2, K=3, W=6, T=48, rho=0.1)
    lam = 0.2 * oracle.lambda_max(X, D)
    A = _toeplitz_design(D, X.shape[1])
    zf = _fista(A, X.reshape(-1), lam).reshape(D.shape[0], -1)
    Z, st, _ = oracle.lgcd(X, D, lam, 1e-12, 3)
    assert st["converged"] == 1
    np.testing.assert_allclose(Z, zf, atol=1e-8)
    Ef = 0.5 * np.sum((X.reshape(-1) - A @ zf.reshape(-1)) ** 2) + lam * np.abs(zf).sum()
    assert abs(oracle.objective(X, D, Z, lam) - Ef) <= 1e-10 * Ef


def scaled_atoms(D, seed, lo=0.3, hi=3.0):
    """The atoms of D rescaled to norms drawn uniformly in [lo, hi], so that the
    division by |D_k|^2 of eq. (pb_coord) is not a division by 1."""
    rng = np.random.default_rng(seed)
    nrm = rng.uniform(lo, hi, size=D.shape[0])
    return D / np.sqrt(np.sum(D * D, axis=(1, 2), keepdims=True)) * nrm[:, None, None]


@pytest.mark.parametrize("seed", [0, 1])
def test_scaled_atoms_explicit_toeplitz_lasso(seed):
    # Atoms of norms in [0.3, 3]: the Lasso of Sec. 2.1 solved by FISTA on the
    # explicit design, and the KKT conditions (Theorem A.1) written from the
    # subgradient of eq. (2) with A^T (x - A z) recomputed from the design.
    X, D, _ = tiny_problem(seed + 10, P=2, K=3, W=6, T=48, rho=0.1)
    D = scaled_atoms(D, seed)
    assert np.ptp(np.sqrt(np.sum(D * D, axis=(1, 2)))) > 0.5
    lam = 0.2 * oracle.lambda_max(X, D)
    A = _toeplitz_design(D, X.shape[1])
    zf = _fista(A, X.reshape(-1), lam, n_iter=200000).reshape(D.shape[0], -1)
    Z, st, _ = oracle.lgcd(X, D, lam, 1e-12, 3)
    assert st["converged"] == 1
    np.testing.assert_allclose(Z, zf, atol=1e-7)
    c = (A.T @ (X.reshape(-1) - A @ Z.reshape(-1))).reshape(Z.shape)  # -grad of the quadratic
    on = Z != 0
    n2 = np.sum(D * D, axis=(1, 2))[:, None] * np.ones_like(Z)
    assert np.all(np.abs(c[on] - lam * np.sign(Z[on])) <= 1e-9 * n2[on] + 1e-9)
    assert np.all(np.abs(c[~on]) <= lam + 1e-9 * n2[~on] + 1e-9)


def test_max_dz_matches_definition_scaled_atoms():
    # The stop test of Sec. 2.1 / Algorithm 3: max over all coordinates of
    # |Sh(beta, lambda) / |D_k|^2 - Z|, with beta from its definition (the
    # replacement operator), at an arbitrary Z and atoms of unequal norms.
    X, D, Zt = tiny_problem(12, P=2, K=3, W=5, T=30, rho=0.3)
    D = scaled_atoms(D, 4)
    rng = np.random.default_rng(5)
    Z = 0.3 * Zt + 0.01 * rng.standard_normal(Zt.shape)
    lam = 0.15 * oracle.lambda_max(X, D)
    B = _beta_by_definition(X, D, Z)
    n2 = np.array([np.sum(D[k] ** 2) for k in range(D.shape[0])])
    dz = np.abs(np.sign(B) * np.maximum(np.abs(B) - lam, 0.0) / n2[:, None] - Z)
    v, k, t = oracle.max_dz(X, D, Z, lam)
    assert abs(v - dz.max()) <= 1e-12 * max(1.0, dz.max())
    assert dz[k, t] == dz.max()


def test_kkt_conditions_at_solution():
    # Coordinate-wise optimality (Theorem A.1) in terms of
    # g = beta - |D_k|^2 Z: |g - lambda sign z| <= |D|^2 eps on the support,
    # |g| <= lambda + |D|^2 eps elsewhere.
    X, D, _ = synth.workload(synth.SMALL, 1)
    lam = 0.1 * oracle.lambda_max(X, D)
    eps = 1e-6
    Z, st, _ = oracle.lgcd(X, D, lam, eps, 4, cap=16)
    n2 = oracle.norms(D)[:, None]
    g = oracle.beta(X, D, Z) - n2 * Z
    on = Z != 0
    assert np.all(np.abs(g[on] - lam * np.sign(Z[on])) <= (n2 * eps * np.ones_like(Z))[on] * (1 + 1e-9))
    assert np.all(np.abs(g[~on]) <= lam + (n2 * eps * np.ones_like(Z))[~on])
    assert oracle.max_dz(X, D, Z, lam)[0] < eps


def test_schedules_reach_the_same_solution():
    # Theorem 1: every schedule converges to the same minimiser; eps-solutions
    # of different schedules agree to the accuracy eps allows.
    X, D, _ = synth.workload(synth.SMALL, 3)
    lam = 0.1 * oracle.lambda_max(X, D)
    ref, _, _ = oracle.lgcd(X, D, lam, 1e-11, 1)
    Eref = oracle.objective(X, D, ref, lam)
    runs = [
        oracle.lgcd(X, D, lam, 1e-6, 4)[0],
        oracle.lgcd(X, D, lam, 1e-6, 4, cap=1)[0],
        oracle.lgcd(X, D, lam, 1e-6, 16, cap=8)[0],
        oracle.lgcd(X, D, lam, 1e-6, 4, schedule=oracle.SCHED_SEQUENCE,
                    seq=synth.segment_sequence(4, 50000, 9))[0],
        oracle.lgcd(X, D, lam, 1e-6, 8, schedule=oracle.SCHED_SEQUENCE,
                    seq=np.arange(8))[0],
    ]
    for Z in runs:
        assert np.max(np.abs(Z - ref)) <= 1e-4
        assert abs(oracle.objective(X, D, Z, lam) - Eref) <= 1e-9 * Eref


def test_h1_coherence_of_generated_dictionaries():
    # H1: |S_{k0,k1}[d]| / (|D_k0| |D_k1|) < 1 away from (k0 = k1, d = 0).
    for w in (synth.SMALL, synth.PAPER):
        _, D, _ = synth.generate(w.P, w.K, w.W, 4 * w.W, w.rho, w.sigma_noise, 0)
        D = D.astype(np.float64)
        S = oracle.s_table(D)
        nrm = np.sqrt(oracle.norms(D))
        C = S / (nrm[:, None, None] * nrm[None, :, None])
        K, W = D.shape[0], D.shape[2]
        C[np.arange(K), np.arange(K), W - 1] = 0.0
        assert np.max(np.abs(C)) < 1.0


def test_h1_ratio_closed_forms():
    """The H1 quantity of Theorem 1 (Sec. 3) on dictionaries with known values:
    one atom [1, 1] / sqrt(2) has S[+-1] = 1/2; an atom and its one-sample shift
    reach the Cauchy-Schwarz bound 1 (H1 fails); two 2-channel atoms whose
    shifted cross-correlations are 1 with squared norms 2 give 1/2."""
    D = np.array([[[1.0, 1.0]]]) / np.sqrt(2.0)
    assert abs(oracle.h1_ratio(D) - 0.5) <= 1e-15
    a, b = 0.6, -0.8
    D = np.array([[[a, b, 0.0]], [[0.0, a, b]]])
    assert abs(oracle.h1_ratio(D) - 1.0) <= 1e-15
    D = np.array([[[1.0, 0.0], [0.0, 1.0]], [[0.0, 1.0], [1.0, 0.0]]])
    assert abs(oracle.h1_ratio(D) - 0.5) <= 1e-15
    assert oracle.h1_ratio(np.array([[[2.0]]])) == 0.0      # W = 1: no shift


def test_h1_ratio_matches_numpy_definition():
    """max over k, l, d != 0 of |sum_p sum_tau D_k[p][tau] D_l[p][tau + d]| /
    (|D_k| |D_l|), formed with numpy.correlate per channel."""
    rng = np.random.default_rng(8)
    for K, P, W in ((3, 2, 5), (4, 1, 7), (2, 3, 1)):
        D = rng.standard_normal((K, P, W))
        best = 0.0
        for k in range(K):
            for l in range(K):
                # numpy.correlate(a, v, 'full')[n] = sum_m a[m + n - (W - 1)] v[m]
                c = sum(np.correlate(D[l, p], D[k, p], "full") for p in range(P))
                nk, nl = np.linalg.norm(D[k]), np.linalg.norm(D[l])
                for d in range(-(W - 1), W):
                    if d != 0:
                        best = max(best, abs(c[d + W - 1]) / (nk * nl))
        assert abs(oracle.h1_ratio(D) - best) <= 1e-13 * max(best, 1e-300) + 1e-300


# ------------------------------------------------- safe screening (Gap Safe)

def _scaled(D, seed, lo=0.3, hi=3.0):
    rng = np.random.default_rng(seed)
    Dn = D / np.sqrt(np.sum(D ** 2, axis=(1, 2), keepdims=True))
    return Dn * rng.uniform(lo, hi, size=D.shape[0])[:, None, None]


def test_gap_safe_closed_form_at_zero():
    """At Z = 0 the residual is X and theta = X / max(lambda, lambda_max):
    gap = |X|^2 / 2 (1 - lambda / lambda_max)^2 for lambda < lambda_max, 0 above;
    above lambda_max every coordinate with |beta| < lambda is screened."""
    X, D, _ = tiny_problem(4)
    D = _scaled(D, 4)
    Z = np.zeros((D.shape[0], X.shape[1] - D.shape[2] + 1))
    lmax = oracle.lambda_max(X, D)
    xx = float(np.sum(X ** 2))
    for f in (0.1, 0.5, 0.9):
        g, r, sc = oracle.gap_safe(X, D, Z, f * lmax)
        ref = 0.5 * xx * (1.0 - f) ** 2
        assert abs(g - ref) <= 1e-12 * xx, (g, ref)
        assert abs(r - np.sqrt(2.0 * ref) / (f * lmax)) <= 1e-9 * r
    g, r, sc = oracle.gap_safe(X, D, Z, 1.5 * lmax)
    assert g <= 1e-12 * xx
    B = oracle.correlate(D, X)
    assert np.array_equal(sc, np.abs(B) / (1.5 * lmax) + r * np.sqrt(oracle.norms(D))[:, None] < 1)
    assert sc.all()


def _numpy_corr(D, R):
    """c_k[t] = sum_p sum_tau D_k[p][tau] R[p][t + tau] with numpy.correlate."""
    K, P, W = D.shape
    return np.array([sum(np.correlate(R[p], D[k, p], "valid") for p in range(P))
                     for k in range(K)])


@pytest.mark.parametrize("seed", [0, 1])
def test_gap_safe_is_safe_and_bounds_the_objective(seed):
    """At iterates of every accuracy: the dual point is feasible (numpy),
    E(Z) - E(Z*) <= gap (weak duality), and every screened coordinate is zero
    in the reference solution (eps_ref = 1e-10) and in the explicit Toeplitz
    Lasso solved by ISTA; atoms of unequal norms."""
    X, D, _ = tiny_problem(10 + seed, P=2, K=3, W=6, T=60, rho=0.06)
    D = _scaled(D, seed)
    K, P, W = D.shape
    L = X.shape[1] - W + 1
    lam = 0.2 * oracle.lambda_max(X, D)
    Zref, st, _ = oracle.lgcd(X, D, lam, 1e-10, 1)
    assert st["converged"] == 1
    Eref = oracle.objective(X, D, Zref, lam)
    # explicit Toeplitz Lasso: columns are the shifted atoms
    A = np.zeros((P * X.shape[1], K * L))
    for k in range(K):
        for t in range(L):
            col = np.zeros((P, X.shape[1]))
            col[:, t:t + W] = D[k]
            A[:, k * L + t] = col.ravel()
    step = 1.0 / np.linalg.norm(A, 2) ** 2
    z = np.zeros(K * L)
    for _ in range(20000):
        v = z - step * (A.T @ (A @ z - X.ravel()))
        z = np.sign(v) * np.maximum(np.abs(v) - step * lam, 0.0)
    Zista = z.reshape(K, L)
    rng = np.random.default_rng(seed)
    n_total = 0
    for eps in (1e-1, 1e-3, 1e-6):
        Z, _, _ = oracle.lgcd(X, D, lam, eps, 1)
        for Zi in (Z, Z + 0.01 * rng.standard_normal(Z.shape) * (Z != 0)):
            g, r, sc = oracle.gap_safe(X, D, Zi, lam)
            R = X - oracle.reconstruct(D, Zi, X.shape[1])
            c = _numpy_corr(D, R)
            sc_ = max(lam, np.abs(c).max())
            assert np.abs(c / sc_).max() <= 1.0 + 1e-12
            assert oracle.objective(X, D, Zi, lam) - Eref <= g * (1 + 1e-9) + 1e-12
            assert not np.any(Zref[sc] != 0)
            assert np.all(np.abs(Zista[sc]) <= 1e-8)
            n_total += int(sc.sum())
    assert n_total > 0


def test_gap_safe_mask_is_the_sphere_test():
    """The screened set is exactly the set of coordinates whose shifted atom
    a (a column of the explicit Toeplitz matrix) keeps |<a, theta'>| < 1 over
    the whole ball around theta of radius sqrt(2 gap) / lambda: the maximum
    over that ball is attained at theta' = theta + r a / |a| (or its mirror),
    evaluated here explicitly; theta, the primal and the dual objectives are
    formed with numpy.  Atoms of unequal norms, iterates of several accuracies."""
    X, D, _ = tiny_problem(21, P=2, K=3, W=6, T=60, rho=0.06)
    D = _scaled(D, 21)
    K, P, W = D.shape
    T = X.shape[1]
    L = T - W + 1
    lam = 0.2 * oracle.lambda_max(X, D)
    A = np.zeros((P * T, K * L))
    for k in range(K):
        for t in range(L):
            col = np.zeros((P, T))
            col[:, t:t + W] = D[k]
            A[:, k * L + t] = col.ravel()
    x = X.ravel()
    n_diff_norm = 0
    for eps in (3e-1, 1e-1, 1e-2, 1e-4):
        Z, _, _ = oracle.lgcd(X, D, lam, eps, 1)
        z = Z.ravel()
        res = x - A @ z
        c = A.T @ res
        sc = max(lam, np.abs(c).max())
        theta = res / sc
        primal = 0.5 * res @ res + lam * np.abs(z).sum()
        dual = 0.5 * x @ x - 0.5 * lam ** 2 * np.sum((theta - x / lam) ** 2)
        r = np.sqrt(2.0 * max(primal - dual, 0.0)) / lam
        g, r_o, mask = oracle.gap_safe(X, D, Z, lam)
        assert abs(g - (primal - dual)) <= 1e-9 * max(1.0, primal)
        for j in range(K * L):
            a = A[:, j]
            na = np.linalg.norm(a)
            top = max(abs(a @ (theta + r * a / na)), abs(a @ (theta - r * a / na)))
            if abs(top - 1.0) < 1e-9:
                continue                      # on the boundary: rounding decides
            assert mask.ravel()[j] == (top < 1.0), (eps, j, top)
            n_diff_norm += (abs(a @ theta) + r < 1.0) != (top < 1.0)
    assert n_diff_norm > 0    # the atom norm changed the decision somewhere


def test_bad_arguments_rejected():
    X, D, _ = tiny_problem(0)
    with pytest.raises(ValueError):
        oracle.lgcd(X, D, 0.0, 1e-6, 1)
    with pytest.raises(ValueError):
        oracle.lgcd(X, D, 1.0, 0.0, 1)
    with pytest.raises(ValueError):        # segments shorter than 2W
        oracle.lgcd(X, D, 1.0, 1e-6, 8)


# ------------------------------------------- Algorithm 2 in lockstep (DICOD)

def test_prop_a2_two_concurrent_updates():
    # Prop. A.2: two coordinates moved from the same Z to their own optimal
    # values change the cost by dE0 + dE1 - S_{k0,k1}[t0 - t1] d0 d1 (each dE
    # of Prop. A.1 measured alone), checked against the objective directly.
    X, D, Zt = tiny_problem(9, P=2, K=3, W=6, T=40, rho=0.2)
    K, P, W = D.shape
    L = Zt.shape[0 + 1]
    lam = 0.1 * oracle.lambda_max(X, D)
    S = oracle.s_table(D)
    n2 = oracle.norms(D)
    rng = np.random.default_rng(3)
    Z = 0.5 * Zt + 0.05 * rng.standard_normal(Zt.shape)
    B = oracle.beta(X, D, Z)
    E0 = oracle.objective(X, D, Z, lam)
    checked = 0
    for _ in range(40):
        k0, k1 = rng.integers(0, K, 2)
        t0 = int(rng.integers(0, L))
        t1 = int(np.clip(t0 + rng.integers(-W + 1, W), 0, L - 1))
        if (k0, t0) == (k1, t1):
            continue
        z0 = oracle.soft_threshold(B[k0, t0], lam) / n2[k0]
        z1 = oracle.soft_threshold(B[k1, t1], lam) / n2[k1]
        d0, d1 = z0 - Z[k0, t0], z1 - Z[k1, t1]
        Za, Zb, Zab = Z.copy(), Z.copy(), Z.copy()
        Za[k0, t0] = z0
        Zb[k1, t1] = z1
        Zab[k0, t0], Zab[k1, t1] = z0, z1
        dE0 = E0 - oracle.objective(X, D, Za, lam)
        dE1 = E0 - oracle.objective(X, D, Zb, lam)
        dE01 = E0 - oracle.objective(X, D, Zab, lam)
        pred = dE0 + dE1 - S[k0, k1, t0 - t1 + W - 1] * d0 * d1
        assert abs(dE01 - pred) <= 1e-9 * max(1.0, abs(dE01)), (k0, t0, k1, t1)
        checked += abs(t0 - t1) > 0 and abs(d0 * d1) > 0
    assert checked > 10


@pytest.mark.parametrize("seed,M,cap", [(0, 4, 1), (1, 4, 3), (2, 8, 1), (3, 5, 0)])
def test_dicod_schedule_cost_identity(seed, M, cap):
    # In a lockstep phase every core picks its update from its own beta; the
    # total cost decrease is the sum of the single-update decreases (Prop. A.1,
    # each on the state its core saw) minus the interference terms of all
    # concurrent pairs of adjacent cores within W (Prop. A.2, every pair).
    X, D, _ = tiny_problem(seed, P=2, K=3, W=6, T=6 * M + 5 + 6 * 6, rho=0.15)
    lam = 0.08 * oracle.lambda_max(X, D)
    Z, st, _ = oracle.lgcd(X, D, lam, 1e-9, M, schedule=oracle.SCHED_DICOD, cap=cap)
    assert st["converged"] == 1
    E0 = oracle.objective(X, D, np.zeros_like(Z), lam)
    E1 = oracle.objective(X, D, Z, lam)
    assert abs((E0 - E1) - (st["dE_sum"] - st["interf_sum"])) <= 1e-9 * (E0 - E1)
    assert st["n_interf"] <= st["n_adjacent"]


def test_dicod_schedule_interferes_and_converges():
    # Short segments make concurrent neighbouring updates interfere; the run
    # still reaches an eps-solution (Theorem 1 under H1), the same optimum as
    # the sequential schedule.
    X, D, _ = tiny_problem(4, P=2, K=3, W=8, T=200, rho=0.1)
    lam = 0.05 * oracle.lambda_max(X, D)
    Zd, sd, _ = oracle.lgcd(X, D, lam, 1e-10, 20, schedule=oracle.SCHED_DICOD, cap=1)
    Zs, ss, _ = oracle.lgcd(X, D, lam, 1e-10, 20, cap=1, colors=3)
    assert sd["converged"] == 1 and sd["n_interf"] > 0
    mdz, _, _ = oracle.max_dz(X, D, Zd, lam)
    assert mdz < 1e-10
    Ed, Es = oracle.objective(X, D, Zd, lam), oracle.objective(X, D, Zs, lam)
    assert abs(Ed - Es) <= 1e-9 * Es
    np.testing.assert_allclose(Zd, Zs, rtol=0, atol=1e-6 * np.abs(Zs).max())


def test_dicod_single_core_is_greedy_cd():
    # M = 1: no neighbour, no message; Algorithm 2 reduces to Algorithm 1.
    X, D, _ = tiny_problem(5, P=2, K=2, W=4, T=30, rho=0.15)
    lam = 0.1 * oracle.lambda_max(X, D)
    Za, sa, ta = oracle.lgcd(X, D, lam, 1e-9, 1, schedule=oracle.SCHED_DICOD, cap=1,
                             trace_cap=200)
    Zb, sb, tb = oracle.lgcd(X, D, lam, 1e-9, 1, cap=1, trace_cap=200)
    assert sa["n_messages"] == 0 and sa["n_interf"] == 0
    np.testing.assert_array_equal(ta[["k0", "t0"]], tb[["k0", "t0"]])
    np.testing.assert_array_equal(Za, Zb)
