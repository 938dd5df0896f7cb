"""Pins of the oracle's propagators: conservation laws, the free-fermion closed
form, a library routine, short-time expansion and the paper's Krylov error bound."""
import numpy as np
import pytest

from oracle import basis as B
from oracle import exact as X
from oracle import freefermion as FF
from oracle import hamiltonian as Hm
from oracle import krylov as K
from oracle import midsize as MS
from oracle import model as M
from workloads import BETA_GOLDEN, random_complex, random_fields


def _setup(L, pbc, jxy=1.0, jz=1.0, h=None):
    N = L // 2
    if h is None:
        h = M.fields(L, 1.5, BETA_GOLDEN, 0.4)
    st = B.sector_states(L, N)
    r0 = int(B.lookup(st, [M.neel_state(L)])[0])
    return N, h, st, r0, Hm.build_dense(L, N, pbc, jxy, jz, h)


def test_norm_energy_conservation_and_time_reversal():
    L = 10
    N, h, st, r0, H = _setup(L, True)
    psi0 = random_complex(len(st), 7)
    psi0 /= np.linalg.norm(psi0)
    t = np.array([0.0, 0.3, 2.0, 11.0])
    psis = X.evolve(H, psi0, t)
    E0 = np.vdot(psi0, H @ psi0).real
    for p in psis:
        assert np.linalg.norm(p) == pytest.approx(1.0, abs=1e-13)
        assert np.vdot(p, H @ p).real == pytest.approx(E0, abs=1e-12)
    # F(-t) = F(t) for a real initial state and real H
    F_p = X.survival_probability(H, r0, t)
    F_m = X.survival_probability(H, r0, -t)
    assert np.allclose(F_p, F_m, atol=1e-14)
    # F(0) = sum_n U[r0, n]^2 is 1 to the orthonormality of the computed
    # eigenvectors, about D * eps = 3e-14 here (and it varies with the number
    # of BLAS threads)
    assert F_p[0] == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("pbc", [False, True])
@pytest.mark.parametrize("L", [6, 8, 10])
def test_free_fermion_determinant_matches_dense(L, pbc):
    h = random_fields(L, 11 + L)
    N, _, st, r0, H = _setup(L, pbc, jxy=1.0, jz=0.0, h=h)
    t = np.linspace(0, 12, 25)
    F_dense = X.survival_probability(H, r0, t)
    F_ff = FF.survival_probability(L, N, pbc, 1.0, h, M.neel_state(L), t)
    assert np.max(np.abs(F_dense - F_ff)) < 1e-12


def test_free_fermion_other_fillings():
    # odd particle number on a ring flips the boundary sign relative to even
    for L, N in [(7, 3), (8, 3), (9, 4)]:
        h = random_fields(L, L)
        st = B.sector_states(L, N)
        s = int(st[len(st) // 3])
        H = Hm.build_dense(L, N, True, 1.0, 0.0, h)
        r0 = int(B.lookup(st, [s])[0])
        t = np.linspace(0, 5, 11)
        assert np.allclose(X.survival_probability(H, r0, t),
                           FF.survival_probability(L, N, True, 1.0, h, s, t), atol=1e-12)


def test_short_time_expansion():
    # F(t) = 1 - beta0^2 t^2 + O(t^4) with beta0 the first Lanczos norm of e_r0
    L = 10
    N, h, st, r0, H = _setup(L, True)
    e = np.zeros(len(st)); e[r0] = 1
    E0 = H[r0, r0]
    beta0sq = np.sum((H @ e - E0 * e) ** 2)
    for t in [1e-3, 3e-3]:
        F = X.survival_probability(H, r0, [t])[0]
        assert (1 - F) / t ** 2 == pytest.approx(beta0sq, rel=1e-4)


def test_expm_multiply_matches_dense():
    L = 12
    N, h, st, r0, H = _setup(L, False)
    t = np.array([0.0, 0.5, 1.7, 6.0])
    Hc = Hm.build_csr(L, N, False, 1.0, 1.0, h)
    psi0 = np.zeros(len(st), complex); psi0[r0] = 1
    a = MS.evolve(Hc, psi0, t)
    b = X.evolve(H, psi0, t)
    assert np.max(np.abs(a - b)) < 1e-12
    assert np.allclose(MS.survival_probability(Hc, r0, t), X.survival_probability(H, r0, t), atol=1e-12)


def test_autocorrelation_simple_cases():
    t = np.linspace(0, 4, 401)
    assert np.allclose(X.autocorrelation(t, np.full_like(t, 0.25)), 0.25)
    C = X.autocorrelation(t, np.exp(-t))
    assert C[-1] == pytest.approx((1 - np.exp(-4)) / 4, rel=1e-5)


def test_krylov_converged_matches_exact():
    L = 10
    N, h, st, r0, H = _setup(L, True)
    psi0 = np.zeros(len(st), complex); psi0[r0] = 1
    dt, steps = 0.1, 20
    psi, F = K.evolve(lambda v: H @ v, psi0, dt, steps, 30, r0=r0)
    t = dt * np.arange(1, steps + 1)
    assert np.max(np.abs(F - X.survival_probability(H, r0, t))) < 1e-12
    assert np.max(np.abs(psi - X.evolve(H, psi0, [dt * steps])[0])) < 1e-11


def test_krylov_projection_is_tridiagonal_real():
    # Hermitian H: the Arnoldi matrix is tridiagonal with real diagonal and
    # positive real subdiagonal (the Lanczos coefficients), alpha_0 = E0.
    L = 10
    N, h, st, r0, H = _setup(L, True)
    psi0 = np.zeros(len(st), complex); psi0[r0] = 1
    V, A, beta0, hn, mu = K.arnoldi(lambda v: H @ v, psi0, 12)
    assert mu == 12
    assert np.allclose(np.triu(A, 2), 0, atol=1e-12)
    assert np.allclose(A.imag, 0, atol=1e-13)
    sub = np.diag(A, -1).real
    assert np.all(sub > 0)
    assert np.allclose(np.diag(A, 1), sub, atol=1e-12)
    assert A[0, 0].real == pytest.approx(H[r0, r0], abs=1e-13)
    assert sub[0] == pytest.approx(0.5 * np.sqrt(L), abs=1e-13)   # all L ring bonds anti-aligned
    assert np.allclose(V.conj().T @ V, np.eye(mu), atol=1e-12)


def test_krylov_breakdown_cases():
    # invariant subspace: an eigenvector gives m_used = 1 and F = 1
    L = 8
    N, h, st, r0, H = _setup(L, True)
    w, U = np.linalg.eigh(H)
    psi, info = K.expm_step(lambda v: H @ v, U[:, 3].astype(complex), 0.7, 30)
    assert info["m_used"] == 1
    assert abs(np.vdot(U[:, 3], psi)) ** 2 == pytest.approx(1.0, abs=1e-14)
    # D < m: the Krylov space is the whole sector and the step is exact
    N4, h4, st4, r04, H4 = _setup(4, True)
    psi0 = np.zeros(6, complex); psi0[r04] = 1
    psi, info = K.expm_step(lambda v: H4 @ v, psi0, 1.3, 30)
    assert info["m_used"] <= 6
    assert np.allclose(psi, X.evolve(H4, psi0, [1.3])[0], atol=1e-13)


def test_krylov_error_within_paper_bound():
    # Sec. 2: the Krylov error behaves like e^(m - t||A||) (t||A||/m)^m once m
    # exceeds t||A||; published forms of this bound carry a constant <= 12.
    L = 10
    N, h, st, r0, H = _setup(L, True)
    normA = np.max(np.abs(np.linalg.eigvalsh(H)))
    psi0 = np.zeros(len(st), complex); psi0[r0] = 1
    checked = 0
    for m in range(4, 24, 2):
        for t in [0.05, 0.1, 0.2, 0.4]:
            if m < t * normA:
                continue
            psi, _ = K.expm_step(lambda v: H @ v, psi0, t, m)
            err = np.linalg.norm(psi - X.evolve(H, psi0, [t])[0])
            assert err <= 12 * K.error_bound(m, t, normA) + 1e-13
            checked += 1
    assert checked > 20


def test_error_bound_is_tight_at_the_edge_of_its_regime():
    # The a-priori bound of Sec. 2 against brute force: a diagonal operator
    # whose 2000 eigenvalues fill [-1, 1] with the Chebyshev density (the
    # spectrum on which polynomials, and so Krylov spaces, approximate the
    # exponential worst) and a flat start vector.  At t ||A|| = m, the edge of
    # the regime m >= t ||A|| in which the bound is stated, the true error of
    # the m-dimensional Krylov step is 0.35-0.45 and the bound must lie above
    # it by less than a factor 5: an overestimate (a flipped sign in the
    # exponent, an extra factor e) fails the upper side, a dropped e^m or a
    # wrong power the lower side.  Inside the regime (t ||A|| = m / 2) the
    # bound must still hold.
    n = 2000
    lam = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    v = np.ones(n) / np.sqrt(n)
    for m in (6, 10, 16, 24):
        for x, lo, hi in ((float(m), 1.0, 5.0), (0.5 * m, 1.0, np.inf)):
            psi, _ = K.expm_step(lambda u: lam * u, v, x, m)
            err = np.linalg.norm(psi - np.exp(-1j * x * lam) * v)
            ratio = K.error_bound(m, x, 1.0) / err
            assert lo <= ratio <= hi, (m, x, err, ratio)
    # the shape e^(m - x) (x / m)^m peaks where m log x - x does, at x = m,
    # with value 1
    for m in (5, 12, 30):
        xs = np.linspace(0.2 * m, 3 * m, 2801)
        vals = np.array([K.error_bound(m, x, 1.0) for x in xs])
        assert abs(xs[np.argmax(vals)] - m) < 3 * (xs[1] - xs[0])
        assert abs(K.error_bound(m, 1.0, float(m)) - 1.0) < 1e-12


def test_saad_estimate_tracks_error():
    L = 10
    N, h, st, r0, H = _setup(L, True)
    psi0 = np.zeros(len(st), complex); psi0[r0] = 1
    # Before roundoff takes over, the estimate bounds the true error from
    # above, and not by more than two orders of magnitude.
    for dt in [0.2, 0.5]:
        for m in [4, 6, 8, 10, 12]:
            psi, info = K.expm_step(lambda v: H @ v, psi0, dt, m)
            err = np.linalg.norm(psi - X.evolve(H, psi0, [dt])[0])
            assert err < info["err_est"] < err * 100


def test_autocorrelation_exact_two_level_closed_form():
    # two sites, one particle, open chain: P(t) = 1 - (jxy/W)^2 sin^2(W t / 2),
    # W = sqrt(jxy^2 + (h1 - h2)^2), so its time average over [0, t] is
    # 1 - (jxy/W)^2 (1/2 - sin(W t) / (2 W t))
    jxy, h = 0.8, np.array([0.9, -0.4])
    Hd = Hm.build_dense(2, 1, False, jxy, 0.3, h)
    W = np.sqrt(jxy ** 2 + (h[0] - h[1]) ** 2)
    t = np.array([1e-9, 0.3, 1.7, 12.0])
    e0 = np.array([1.0, 0.0])
    ref = 1.0 - (jxy / W) ** 2 * (0.5 - np.sin(W * t) / (2 * W * t))
    assert np.max(np.abs(X.autocorrelation_exact(Hd, e0, t) - ref)) < 1e-12


def test_autocorrelation_exact_limits_and_trapezoid():
    L = 8
    hf = M.fields(L, 1.2, BETA_GOLDEN, 0.7)
    Hd = Hm.build_dense(L, L // 2, True, 1.0, 1.0, hf)
    eig = X.eig(Hd)
    rng = np.random.default_rng(3)
    psi0 = rng.standard_normal(len(Hd)) + 1j * rng.standard_normal(len(Hd))
    psi0 /= np.linalg.norm(psi0)
    # t -> 0: C = P(0) = 1
    assert abs(X.autocorrelation_exact(Hd, psi0, [1e-10], eig)[0] - 1.0) < 1e-12
    # long times: C -> sum_n w_n^2 (inverse participation ratio), within O(1/t)
    c = eig[1].T @ psi0
    ipr = float(np.sum(np.abs(c) ** 4))
    T = 1e6
    assert abs(X.autocorrelation_exact(Hd, psi0, [T], eig)[0] - ipr) < 1e-4
    # the trapezoid rule on exact P converges to the closed form as dt^2
    errs = []
    for dt in (0.02, 0.01):
        t = dt * np.arange(0, int(round(3.0 / dt)) + 1)
        P = np.array([X.overlap_probability(psi0, v) for v in X.evolve(Hd, psi0, t, eig)])
        Ct = X.autocorrelation(t, P)
        errs.append(abs(Ct[-1] - X.autocorrelation_exact(Hd, psi0, [3.0], eig)[0]))
    assert errs[0] < 1e-4 and 3.0 < errs[0] / errs[1] < 5.0


@pytest.mark.parametrize("L,pbc,jz", [(10, True, 1.0), (12, False, 0.7)])
def test_moment_expansion_matches_dense(L, pbc, jz):
    # the short-time expansion used at full size (tests/moments.py) against
    # the dense exact propagation, for the Neel amplitude and states 1-3 hops away
    import moments as MO
    N = L // 2
    h = M.fields(L, 1.5, BETA_GOLDEN, 0.4)
    Hd = Hm.build_dense(L, N, pbc, 1.0, jz, h)
    states = B.sector_states(L, N)
    neel = M.neel_state(L)
    r0 = int(B.lookup(states, [neel])[0])
    e0 = np.zeros(len(states))
    e0[r0] = 1.0
    others = [neel ^ 0b11, neel ^ 0b1100 ^ (0b11 << 6), neel ^ (0b11 << 2) ^ (0b11 << 4) ^ (0b11 << 8)]
    for t in (0.04, 0.1):
        K = 18
        assert MO.remainder_bound(L, pbc, 1.0, jz, h, t, K) < 1e-13
        psi = X.evolve(Hd, e0, [t])[0]
        pn = MO.powers(neel, K // 2, L, pbc, 1.0, jz, h)
        assert abs(MO.taylor_amplitude(pn, pn, t, K) - psi[r0]) < 1e-13
        for s in others:
            ps = MO.powers(s, K // 2, L, pbc, 1.0, jz, h)
            got = MO.taylor_amplitude(ps, pn, t, K)
            assert abs(got - psi[int(B.lookup(states, [s])[0])]) < 1e-13, (L, t, s)
    # too few powers for the order is refused
    with pytest.raises(ValueError):
        MO.taylor_amplitude(pn[:3], pn[:3], 0.1, 5)
