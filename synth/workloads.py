"""Seeded synthetic workloads drawn from the rank-constrained SCM generative model.

This module only *samples inputs*.  It contains none of the estimation
arithmetic (no E-step, no M-step, no accelerated rule, no extraction): both
the FP64 oracle (``oracle/``) and the GPU library consume the arrays it
returns, and neither of them is imported here.

Generative model (Sec. II-B-1, eqs. (2)-(10)):

    x_ij = a_i s_ij + u_ij,   s_ij ~ N_c(0, r^h_ij),
    u_ij ~ N_c(0, r^u_ij (R'_i + lambda_i b_i b_i^H)),

with R'_i Hermitian PSD of rank M-1, b_i its unit null vector and
lambda_i > 0.  Draws are exact: u_ij = sqrt(r^u_ij) (V_i z1 + sqrt(lambda_i) b_i z2)
with R'_i = V_i V_i^H, so the true dry target s_ij is returned alongside x.

Randomness: one ``numpy.random.SeedSequence(SEED, spawn_key=(config, utterance, i))``
stream per frequency row, consumed in a fixed order (per-frequency spatial
parameters first, then per-bin values), so any frequency row can be
regenerated on its own and equals the same row of the full instance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

SEED = 190801964

# Table 2 of the paper: prior shape/scale and STFT settings.
ALPHA = 1.1
BETA = 1e-16
FS = 16000.0
SOUND_SPEED = 343.0
MIC_SPACING = 0.05
DIAG_LOADING = 1e-3


@dataclass
class Problem:
    """One utterance: observations plus the fixed spatial model (paper notation)."""

    x: np.ndarray  # complex64 [I, J, M]
    a: np.ndarray  # complex128 [I, M]      steering vector a_i
    Rp: np.ndarray  # complex128 [I, M, M]  rank-(M-1) SCM R'_i
    b: np.ndarray  # complex128 [I, M]      unit null vector b_i of R'_i
    s_true: Optional[np.ndarray] = None  # complex64 [I, J] true dry target
    rh_true: Optional[np.ndarray] = None  # float64 [I, J]
    ru_true: Optional[np.ndarray] = None  # float64 [I, J]
    lam_true: Optional[np.ndarray] = None  # float64 [I]
    freqs: Optional[np.ndarray] = None  # frequency indices of the rows held
    meta: dict = field(default_factory=dict)

    @property
    def I(self) -> int:  # noqa: E743 - paper notation
        return self.x.shape[0]

    @property
    def J(self) -> int:
        return self.x.shape[1]

    @property
    def M(self) -> int:
        return self.x.shape[2]


def _rng(config: int, utterance: int, freq: int) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED, spawn_key=(int(config), int(utterance), int(freq)))
    return np.random.Generator(np.random.PCG64(ss))


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Circular complex Gaussian CN(0, 1) samples (unit total variance)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def random_spatial(rng: np.random.Generator, M: int):
    """Per-frequency spatial model of the random recipe.

    a_i ~ CN(0, I) normalised to unit norm; V ~ CN M x (M-1); R' = V V^H;
    b = unit vector orthogonal to range(V) (last column of a complete QR);
    lambda_true ~ U(0.1, 1).
    """
    a = _cn(rng, M)
    a = a / np.linalg.norm(a)
    V = _cn(rng, (M, M - 1))
    Q, _ = np.linalg.qr(V, mode="complete")
    b = Q[:, M - 1].copy()
    b = b / np.linalg.norm(b)
    lam = rng.uniform(0.1, 1.0)
    Rp = V @ V.conj().T
    return a, V, Rp, b, lam


def sinc_coherence(M: int, f: float, spacing: float = MIC_SPACING, c: float = SOUND_SPEED):
    """Diffuse-field coherence of an M-mic uniform linear array at frequency f (Hz).

    Gamma_pq = sin(w)/w with w = 2 pi f d_pq / c (numpy.sinc is the normalised sinc).
    """
    pos = spacing * np.arange(M)
    d = np.abs(pos[:, None] - pos[None, :])
    return np.sinc(2.0 * f * d / c).astype(np.complex128)


def sinc_spatial(M: int, f: float, loading: float = DIAG_LOADING):
    """Split the loaded diffuse coherence into (V, R', b, lambda_true).

    Gamma + loading*I is eigendecomposed; R' keeps the top M-1 eigenpairs,
    b is the bottom eigenvector and lambda_true the bottom eigenvalue.
    """
    G = sinc_coherence(M, f) + loading * np.eye(M)
    w, U = np.linalg.eigh(G)
    lam = float(w[0])
    b = U[:, 0].copy()
    V = U[:, 1:] * np.sqrt(w[1:])[None, :]
    Rp = V @ V.conj().T
    return V, Rp, b, lam


def _draw_row(rng, a, V, b, lam, J):
    M = a.shape[0]
    rh = rng.gamma(0.5, 1.0, size=J)
    ru = rng.gamma(2.0, 0.5, size=J)
    z0 = _cn(rng, J)
    z1 = _cn(rng, (J, M - 1))
    z2 = _cn(rng, J)
    s = np.sqrt(rh) * z0
    u = np.sqrt(ru)[:, None] * (z1 @ V.T + np.sqrt(lam) * z2[:, None] * b[None, :])
    x = s[:, None] * a[None, :] + u
    return x, s, rh, ru


def make_problem(M: int, I: int, J: int, *, config: int = 100, utterance: int = 0,
                 spatial: str = "random", freqs: Optional[Sequence[int]] = None,
                 n_fft: Optional[int] = None, with_truth: bool = True) -> Problem:
    """Draw one utterance.

    spatial="random": the random recipe per frequency (a, V, b, lambda_true).
    spatial="sinc":   a random unit-norm, (R', b, lambda_true) from the loaded
                      sinc coherence at f_i = i fs / n_fft (n_fft = 2(I-1)).
    ``freqs`` selects a subset of the I frequency rows (exactly the rows of the
    full instance).
    """
    if M < 2:
        raise ValueError("M must be >= 2 (R' has rank M-1 >= 1)")
    if freqs is None:
        freqs = np.arange(I)
    freqs = np.asarray(freqs, dtype=np.int64)
    if n_fft is None:
        n_fft = max(2 * (I - 1), 2)
    n = len(freqs)
    x = np.empty((n, J, M), np.complex64)
    s_true = np.empty((n, J), np.complex64)
    rh_t = np.empty((n, J))
    ru_t = np.empty((n, J))
    a_all = np.empty((n, M), np.complex128)
    Rp_all = np.empty((n, M, M), np.complex128)
    b_all = np.empty((n, M), np.complex128)
    lam_all = np.empty(n)
    for r, i in enumerate(freqs):
        rng = _rng(config, utterance, int(i))
        if spatial == "random":
            a, V, Rp, b, lam = random_spatial(rng, M)
        elif spatial == "sinc":
            a = _cn(rng, M)
            a = a / np.linalg.norm(a)
            V, Rp, b, lam = sinc_spatial(M, float(i) * FS / n_fft)
        else:
            raise ValueError(spatial)
        xr, sr, rhr, rur = _draw_row(rng, a, V, b, lam, J)
        x[r] = xr
        s_true[r] = sr
        rh_t[r] = rhr
        ru_t[r] = rur
        a_all[r] = a
        Rp_all[r] = Rp
        b_all[r] = b
        lam_all[r] = lam
    p = Problem(x=x, a=a_all, Rp=Rp_all, b=b_all, freqs=freqs,
                meta=dict(M=M, I_full=I, J=J, config=config, utterance=utterance,
                          spatial=spatial, n_fft=n_fft))
    if with_truth:
        p.s_true, p.rh_true, p.ru_true, p.lam_true = s_true, rh_t, ru_t, lam_all
    return p


def make_bss_problem(M: int, I: int, J: int, *, config: int = 600, target: int = 0,
                     perturb: float = 0.0, freqs: Optional[Sequence[int]] = None) -> dict:
    """Determined mixture x_ij = A_i s_ij (eq. (1)) with one target and M-1 noise sources.

    A_i ~ CN(0, I) (M x M); the demixing matrix is W_i = A_i^{-1} (I + perturb E_i)
    with E_i ~ CN(0, I) (perturb = 0: a perfect separation).  s_target ~ CN(0, r),
    r ~ Gamma(0.5, 1); noise sources ~ CN(0, r), r ~ Gamma(2, 0.5).
    Returns dict(x complex64 [I, J, M], W complex128 [I, M, M], A, s complex128
    [I, J, M], target).
    """
    if freqs is None:
        freqs = np.arange(I)
    freqs = np.asarray(freqs, dtype=np.int64)
    n = len(freqs)
    x = np.empty((n, J, M), np.complex64)
    W = np.empty((n, M, M), np.complex128)
    A_all = np.empty((n, M, M), np.complex128)
    s_all = np.empty((n, J, M), np.complex128)
    for r, i in enumerate(freqs):
        rng = _rng(config, 0, int(i))
        A = _cn(rng, (M, M))
        E = _cn(rng, (M, M))
        pw = np.where(np.arange(M) == target, rng.gamma(0.5, 1.0, (J, M)),
                      rng.gamma(2.0, 0.5, (J, M)))
        s = np.sqrt(pw) * _cn(rng, (J, M))
        x[r] = s @ A.T
        W[r] = np.linalg.inv(A) @ (np.eye(M) + perturb * E)
        A_all[r] = A
        s_all[r] = s
    return dict(x=x, W=W, A=A_all, s=s_all, target=int(target), freqs=freqs)


# --- the five named workloads -------------------------------------------------

WORKLOADS = {
    0: dict(name="random-M2", M=2, I=257, J=250, K=20, spatial="random"),
    1: dict(name="sinc-M4", M=4, I=513, J=1000, K=20, spatial="sinc"),
    2: dict(name="batch64-ragged", U=64, I=513, K=20, spatial="random",
            J_range=(200, 4000), M_choices=(2, 4, 6)),
    3: dict(name="sinc-M4-adjoint", M=4, I=513, J=1000, K=10, spatial="sinc"),
    4: dict(name="sinc-M8-large", M=8, I=1025, J=8000, K=30, spatial="sinc"),
}


def config(cid: int, freqs: Optional[Sequence[int]] = None, with_truth: bool = True) -> Problem:
    """Single-utterance workload ``cid`` in {0, 1, 3, 4} (config 3 reuses config 1's data)."""
    c = WORKLOADS[cid]
    if cid == 2:
        raise ValueError("config 2 is a batch: use batch_shapes()/batch_utterance()")
    seed_cfg = 1 if cid == 3 else cid
    p = make_problem(c["M"], c["I"], c["J"], config=seed_cfg, spatial=c["spatial"],
                     freqs=freqs, with_truth=with_truth)
    p.meta.update(K=c["K"], name=c["name"], cid=cid)
    return p


def batch_shapes(U: int = 64, J_range=(200, 4000), M_choices=(2, 4, 6), cid: int = 2):
    """Per-utterance (J_u, M_u) of the ragged batch, from an utterance-level stream."""
    Js, Ms = [], []
    for u in range(U):
        rng = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(SEED, spawn_key=(int(cid), int(u), 1 << 20))))
        Js.append(int(rng.integers(J_range[0], J_range[1] + 1)))
        Ms.append(int(M_choices[int(rng.integers(0, len(M_choices)))]))
    return Js, Ms


def batch_utterance(u: int, I: int = 513, freqs=None, cid: int = 2, with_truth: bool = False,
                    J_range=(200, 4000), M_choices=(2, 4, 6), U: int = 64) -> Problem:
    Js, Ms = batch_shapes(U, J_range, M_choices, cid)
    p = make_problem(Ms[u], I, Js[u], config=cid, utterance=u, spatial="random",
                     freqs=freqs, with_truth=with_truth)
    p.meta.update(K=WORKLOADS[2]["K"], name=WORKLOADS[2]["name"], cid=cid)
    return p
