"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a second, independently written
statement of the same iteration, generic Gaussian conditioning, numerical
maximisation of the Q function, a textbook closed form, an invariance of the
model, or the constants the paper prints.
"""
import json
import os

import numpy as np
import pytest

from oracle import accel, bruteforce, extract, first_stage, naive, objective
from oracle.linalg import herm, pinv_rank
from synth import ALPHA, BETA, make_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(b), 1e-300)))


def _nrel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# --- the paper's algebra (eqs. (24)-(26), (35)-(38), (40)-(44)) on random inputs ----------

def _rand_model(rng, M):
    a = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    V = rng.standard_normal((M, M - 1)) + 1j * rng.standard_normal((M, M - 1))
    Q, _ = np.linalg.qr(V, mode="complete")
    b = Q[:, -1]
    Rp = V @ V.conj().T
    x = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return a, Rp, b, x


@pytest.mark.parametrize("M", [2, 3, 5, 8])
def test_pseudoinverse_expansion_eq26(M):
    rng = np.random.default_rng(M)
    a, Rp, b, x = _rand_model(rng, M)
    lam = 0.37
    lhs = np.linalg.inv(Rp + lam * np.outer(b, b.conj()))
    rhs = pinv_rank(Rp, M - 1) + np.outer(b, b.conj()) / lam
    assert _rel(rhs, lhs) < 1e-10
    # numpy's SVD-based pseudoinverse agrees with the eigen-based one
    assert np.allclose(pinv_rank(Rp, M - 1), np.linalg.pinv(Rp, rcond=1e-10, hermitian=True),
                       rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("M", [2, 4, 7])
def test_sherman_morrison_and_scalar_identities(M):
    rng = np.random.default_rng(10 + M)
    a, Rp, b, x = _rand_model(rng, M)
    lam_t, rh_t, ru_t = 0.8, 0.6, 1.7
    R_t = Rp + lam_t * np.outer(b, b.conj())
    Rx = rh_t * np.outer(a, a.conj()) + ru_t * R_t
    Rt_inv = np.linalg.inv(R_t)
    rho_aa = np.real(a.conj() @ Rt_inv @ a)
    rho_ax = a.conj() @ Rt_inv @ x
    g = rh_t / (ru_t + rh_t * rho_aa)
    sm = (Rt_inv - g * np.outer(Rt_inv @ a, a.conj() @ Rt_inv)) / ru_t          # eq. (25)
    assert _rel(sm, np.linalg.inv(Rx)) < 1e-10
    assert abs(a.conj() @ sm @ a - rho_aa / (ru_t + rh_t * rho_aa)) < 1e-12         # eq. (36)
    assert abs(a.conj() @ sm @ x - rho_ax / (ru_t + rh_t * rho_aa)) < 1e-12         # eq. (37)
    s_ab = a.conj() @ b
    s_bx = b.conj() @ x
    assert abs(b.conj() @ R_t @ sm @ R_t @ b - (lam_t - g * abs(s_ab) ** 2) / ru_t) < 1e-11  # eq. (41)
    assert abs(b.conj() @ R_t @ sm @ x - (s_bx - g * s_ab.conj() * rho_ax) / ru_t) < 1e-11  # eq. (42)


# --- two independent statements of one iteration agree ---------------------------------------

@pytest.mark.parametrize("M,spatial", [(2, "random"), (3, "random"), (4, "sinc"),
                                        (6, "random"), (8, "sinc")])
def test_naive_equals_accelerated(M, spatial):
    p = make_problem(M, 5, 30, config=201, spatial=spatial, n_fft=64)
    st = accel.init_state(p.I, p.J)
    rn = naive.run(p.x, p.a, p.Rp, p.b, *st, 20, ALPHA, BETA)
    ra = accel.run(p.x, p.a, p.Rp, p.b, *st, 20, ALPHA, BETA)
    r1 = first_stage.run(p.x, p.a, p.Rp, p.b, *st, 20, ALPHA, BETA)
    for q in range(3):
        assert _nrel(ra[q], rn[q]) < 1e-10
        assert _nrel(r1[q], rn[q]) < 1e-10


# --- E-step by generic Gaussian conditioning --------------------------------------------------

@pytest.mark.parametrize("M", [2, 4, 6])
def test_estep_matches_gaussian_conditioning(M):
    p = make_problem(M, 2, 6, config=202)
    rng = np.random.default_rng(3)
    for i in range(p.I):
        rh_t = rng.gamma(1.0, 1.0, p.J)
        ru_t = rng.gamma(2.0, 0.5, p.J)
        lam_t = 0.45
        R_t, h_hat, U_hat = naive.estep(p.x[i].astype(np.complex128), p.a[i], p.Rp[i], p.b[i],
                                        rh_t, ru_t, lam_t)
        for j in range(p.J):
            for route in (bruteforce.estep_joint, bruteforce.estep_precision):
                hb, Ub, _ = route(p.x[i, j].astype(np.complex128), p.a[i], R_t, rh_t[j], ru_t[j])
                assert abs(h_hat[j] - hb) <= 1e-10 * abs(hb)
                assert np.max(np.abs(U_hat[j] - Ub)) <= 1e-10 * np.max(np.abs(Ub))


# --- M-step by numerical maximisation of Q ----------------------------------------------------

@pytest.mark.parametrize("M", [2, 3, 5])
def test_mstep_matches_numeric_argmax(M):
    p = make_problem(M, 2, 5, config=203)
    rng = np.random.default_rng(4)
    for i in range(p.I):
        rh_t = rng.gamma(1.0, 1.0, p.J)
        ru_t = rng.gamma(2.0, 0.5, p.J)
        _, h_hat, U_hat = naive.estep(p.x[i].astype(np.complex128), p.a[i], p.Rp[i], p.b[i],
                                      rh_t, ru_t, 0.7)
        rh, lam, ru = naive.mstep(p.Rp[i], p.b[i], ru_t, h_hat, U_hat, ALPHA, BETA)
        rhb, lamb, rub = bruteforce.mstep_numeric(p.Rp[i], p.b[i], ru_t, h_hat, U_hat, ALPHA, BETA)
        assert _rel(rh, rhb) < 1e-6
        assert abs(lam - lamb) < 1e-6 * lamb
        assert _rel(ru, rub) < 1e-6


# --- whole-iteration properties ---------------------------------------------------------------

@pytest.mark.parametrize("M,spatial", [(2, "random"), (4, "sinc"), (5, "random")])
def test_posterior_never_decreases_map(M, spatial):
    p = make_problem(M, 4, 25, config=204, spatial=spatial, n_fft=16)
    st = accel.init_state(p.I, p.J)
    hist = accel.run(p.x, p.a, p.Rp, p.b, *st, 40, ALPHA, BETA, history=True)
    f = [objective.nlp(p.x, p.a, p.Rp, p.b, *h, ALPHA, BETA) for h in hist]
    d = np.diff(f)
    assert np.all(d <= 1e-9 * np.abs(np.array(f[1:]))), d.max()
    assert f[-1] < f[0]


def test_likelihood_never_decreases_ml_mode():
    # alpha = -1, beta = 0 removes the prior: plain EM on the likelihood.
    p = make_problem(3, 4, 25, config=205)
    st = accel.init_state(p.I, p.J)
    hist = accel.run(p.x, p.a, p.Rp, p.b, *st, 40, -1.0, 0.0, history=True)
    f = [objective.nll(p.x, p.a, p.Rp, p.b, *h) for h in hist]
    assert np.all(np.diff(f) <= 1e-9 * np.abs(np.array(f[1:])))


def test_positivity_and_psd():
    p = make_problem(4, 6, 30, config=206, spatial="sinc", n_fft=10)
    st = accel.init_state(p.I, p.J)
    hist = accel.run(p.x, p.a, p.Rp, p.b, *st, 30, ALPHA, BETA, history=True)
    for rh, ru, lam in hist[1:]:
        assert np.all(rh >= BETA / (ALPHA + 2.0) * (1 - 1e-12))
        assert np.all(ru > 0) and np.all(lam > 0)
        S = objective.sigma(p.a, p.Rp, p.b, rh, ru, lam)
        assert np.allclose(S, herm(S))
        assert np.all(np.linalg.eigvalsh(S) > 0)


def test_target_free_limit_is_ml_scale():
    """r~h -> 0: u = x, so lambda -> mean |b^H x|^2 / r~u and r^u -> x^H R^{-1} x / M."""
    p = make_problem(4, 3, 20, config=207)
    rh0 = np.full((p.I, p.J), 1e-30)
    ru0 = np.random.default_rng(5).gamma(2.0, 0.5, (p.I, p.J))
    lam0 = np.full(p.I, 0.6)
    rh, ru, lam = accel.run(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0, 1, ALPHA, BETA)
    x = p.x.astype(np.complex128)
    lam_ml = np.mean(np.abs(np.einsum("im,ijm->ij", p.b.conj(), x)) ** 2 / ru0, axis=1)
    assert _rel(lam, lam_ml) < 1e-12
    R = p.Rp + lam[:, None, None] * np.einsum("im,in->imn", p.b, p.b.conj())
    q = np.einsum("ijm,ijm->ij", x.conj(),
                  np.linalg.solve(R[:, None], x[..., None])[..., 0]).real
    assert _rel(ru, q / p.M) < 1e-10


def test_decoupled_scalar_case_closed_form():
    """a = e1, b = e2, R' = diag(c, 0): the model splits into two scalar problems.

    s | x1 is the textbook scalar Gaussian posterior with prior variance r~h and
    noise variance r~u c; u2 = x2 exactly.
    """
    rng = np.random.default_rng(6)
    J, c, lam_t = 12, 0.7, 0.4
    a = np.array([[1.0, 0.0]], np.complex128)
    b = np.array([[0.0, 1.0]], np.complex128)
    Rp = np.array([[[c, 0.0], [0.0, 0.0]]], np.complex128)
    x = (rng.standard_normal((1, J, 2)) + 1j * rng.standard_normal((1, J, 2))).astype(np.complex64)
    rh_t = rng.gamma(1.0, 1.0, (1, J))
    ru_t = rng.gamma(2.0, 0.5, (1, J))
    x1 = x[0, :, 0].astype(np.complex128)
    x2 = x[0, :, 1].astype(np.complex128)
    n = ru_t[0] * c
    mean = rh_t[0] * x1 / (rh_t[0] + n)
    var = rh_t[0] * n / (rh_t[0] + n)
    h_hat = var + np.abs(mean) ** 2
    Eu1 = var + np.abs(x1 - mean) ** 2
    rh_exp = (h_hat + BETA) / (ALPHA + 2.0)
    lam_exp = np.mean(np.abs(x2) ** 2 / ru_t[0])
    ru_exp = 0.5 * (Eu1 / c + np.abs(x2) ** 2 / lam_exp)
    for mod in (naive, accel):
        rh, ru, lam = mod.run(x, a, Rp, b, rh_t, ru_t, np.array([lam_t]), 1, ALPHA, BETA)
        assert _rel(rh[0], rh_exp) < 1e-12
        assert abs(lam[0] - lam_exp) < 1e-12 * lam_exp
        assert _rel(ru[0], ru_exp) < 1e-12


def test_fixed_point_is_stationary():
    """Many iterations on a tiny input reach a stationary point of the NLP."""
    p = make_problem(2, 1, 6, config=208)
    st = accel.init_state(p.I, p.J)
    rh, ru, lam = accel.run(p.x, p.a, p.Rp, p.b, *st, 20000, ALPHA, BETA)
    theta = np.concatenate([np.log(rh).ravel(), np.log(ru).ravel(), np.log(lam)])
    n = p.J

    def f(t):
        return objective.nlp(p.x, p.a, p.Rp, p.b, np.exp(t[:n])[None], np.exp(t[n:2 * n])[None],
                             np.exp(t[2 * n:]), ALPHA, BETA)
    g = np.zeros_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = 1e-5
        g[k] = (f(theta + e) - f(theta - e)) / 2e-5
    # compare with the gradient at the start, which is O(1) per coordinate
    assert np.max(np.abs(g)) < 1e-4


def test_extraction_is_posterior_mean():
    p = make_problem(3, 2, 8, config=209)
    rng = np.random.default_rng(7)
    rh = rng.gamma(1.0, 1.0, (p.I, p.J))
    ru = rng.gamma(2.0, 0.5, (p.I, p.J))
    lam = np.array([0.3, 0.9])
    sh = extract.s_hat(p.x, p.a, p.Rp, p.b, rh, ru, lam)
    for i in range(p.I):
        R = p.Rp[i] + lam[i] * np.outer(p.b[i], p.b[i].conj())
        for j in range(p.J):
            _, _, m = bruteforce.estep_joint(p.x[i, j].astype(np.complex128), p.a[i], R,
                                             rh[i, j], ru[i, j])
            assert abs(sh[i, j] - m) < 1e-12 * max(abs(m), 1e-30)


def test_spatial_image_is_posterior_mean_of_the_image():
    """h_hat = a s_hat is E[a s | x]: (1) a times the posterior mean of s from generic Gaussian
    conditioning of [s; u; x]; (2) the complement of the posterior mean of the noise image,
    E[u | x] = r^u R Sigma^{-1} x (cov(u, x) = r^u R), so h_hat + E[u | x] = x.  A conjugated
    or dropped a, or a transposed product, fails one of the two."""
    p = make_problem(4, 2, 6, config=213)
    rng = np.random.default_rng(11)
    rh = rng.gamma(1.0, 1.0, (p.I, p.J))
    ru = rng.gamma(2.0, 0.5, (p.I, p.J))
    lam = np.array([0.4, 1.7])
    img = extract.spatial_image(p.x, p.a, p.Rp, p.b, rh, ru, lam)
    assert img.shape == (p.I, p.J, p.M)
    for i in range(p.I):
        R = p.Rp[i] + lam[i] * np.outer(p.b[i], p.b[i].conj())
        for j in range(p.J):
            x = p.x[i, j].astype(np.complex128)
            _, _, m = bruteforce.estep_joint(x, p.a[i], R, rh[i, j], ru[i, j])
            assert np.max(np.abs(img[i, j] - m * p.a[i])) < 1e-12 * np.linalg.norm(x)
            S = rh[i, j] * np.outer(p.a[i], p.a[i].conj()) + ru[i, j] * R
            u_mean = ru[i, j] * R @ np.linalg.solve(S, x)
            assert np.max(np.abs(img[i, j] + u_mean - x)) < 1e-12 * np.linalg.norm(x)


# --- invariances ------------------------------------------------------------------------------

def test_b_phase_invariance():
    p = make_problem(4, 3, 20, config=210)
    st = accel.init_state(p.I, p.J)
    r0 = accel.run(p.x, p.a, p.Rp, p.b, *st, 10, ALPHA, BETA)
    ph = np.exp(1j * np.array([0.3, -2.0, 1.1]))[:, None]
    r1 = accel.run(p.x, p.a, p.Rp, p.b * ph, *st, 10, ALPHA, BETA)
    for q in range(3):
        assert _rel(r1[q], r0[q]) < 1e-12


def test_frequency_and_frame_permutation():
    p = make_problem(3, 4, 16, config=211)
    st = accel.init_state(p.I, p.J)
    r0 = accel.run(p.x, p.a, p.Rp, p.b, *st, 8, ALPHA, BETA)
    fi = np.array([2, 0, 3, 1])
    fj = np.random.default_rng(8).permutation(p.J)
    r1 = accel.run(p.x[fi][:, fj], p.a[fi], p.Rp[fi], p.b[fi], *st, 8, ALPHA, BETA)
    assert _rel(r1[0], r0[0][fi][:, fj]) < 1e-12
    assert _rel(r1[1], r0[1][fi][:, fj]) < 1e-12
    assert _rel(r1[2], r0[2][fi]) < 1e-12


def test_resume_equals_uninterrupted():
    p = make_problem(4, 3, 20, config=212)
    st = accel.init_state(p.I, p.J)
    r7 = accel.run(p.x, p.a, p.Rp, p.b, *st, 7, ALPHA, BETA)
    r12 = accel.run(p.x, p.a, p.Rp, p.b, *r7, 5, ALPHA, BETA)
    r12b = accel.run(p.x, p.a, p.Rp, p.b, *st, 12, ALPHA, BETA)
    for q in range(3):
        assert np.array_equal(r12[q], r12b[q])


# --- constants the paper prints ----------------------------------------------------------------

def test_paper_constants_golden():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        g = json.load(f)
    assert ALPHA == g["prior"]["alpha"] and BETA == g["prior"]["beta"]
    n_fft = int(g["stft"]["fs_hz"] * g["stft"]["window_ms"] / 1000)
    assert n_fft // 2 + 1 == g["worked_count"]["I"] == 513
    w = g["worked_count"]
    assert w["I"] * w["J"] == w["inversions_per_iteration"]
