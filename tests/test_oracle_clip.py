"""Pins of the oracle's eigenvalue clipping (paper Sec. IV-B, eq. 7)."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "clip_2x2.json")


def test_clip_golden_worked_examples(orc):
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        out = orc.psd_clip(np.array(c["H"]), c["eps"])
        np.testing.assert_allclose(out, np.array(c["Q_psd"]), rtol=1e-14, atol=1e-15)


def test_clip_2x2_closed_form(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b, c = rng.normal(size=3)
        eps = 0.1
        H = np.array([[a, b], [b, c]])
        # closed-form eigenpairs of a symmetric 2x2
        mu = 0.5 * (a + c) + np.array([-1, 1]) * np.hypot(0.5 * (a - c), b)
        out = np.zeros((2, 2))
        for lam in mu:
            v = np.array([b, lam - a]) if abs(b) > 1e-12 else (np.array([1.0, 0]) if abs(lam - a) < abs(lam - c) else np.array([0, 1.0]))
            v /= np.linalg.norm(v)
            out += max(lam, eps) * np.outer(v, v)
        np.testing.assert_allclose(orc.psd_clip(H, eps), out, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12])
def test_clip_matches_numpy_eigh_reconstruction(orc, n):
    rng = np.random.default_rng(n)
    for _ in range(10):
        G = rng.normal(size=(n, n))
        H = 0.5 * (G + G.T)
        eps = 0.05
        w, V = np.linalg.eigh(H)
        ref = V @ np.diag(np.maximum(w, eps)) @ V.T
        out = orc.psd_clip(H, eps)
        np.testing.assert_allclose(out, ref, atol=1e-12)
        # properties: symmetric, spectrum >= eps, idempotent, identity on PSD>=eps
        assert np.array_equal(out, out.T)
        assert np.linalg.eigvalsh(out).min() >= eps * (1 - 1e-10)
        np.testing.assert_allclose(orc.psd_clip(out, eps), out, atol=1e-12)
        S = G @ G.T + eps * np.eye(n)
        np.testing.assert_allclose(orc.psd_clip(S, eps), S, atol=1e-12 * np.abs(S).max())


def test_clip_repeated_eigenvalues_is_unique(orc):
    # clip is a spectral function: with a repeated eigenvalue the eigenvectors
    # are not unique but the result is.
    Qm, _ = np.linalg.qr(np.random.default_rng(7).normal(size=(4, 4)))
    H = Qm @ np.diag([-1.0, -1.0, 2.0, 2.0]) @ Qm.T
    ref = Qm @ np.diag([0.3, 0.3, 2.0, 2.0]) @ Qm.T
    np.testing.assert_allclose(orc.psd_clip(H, 0.3), ref, atol=1e-13)


def test_jacobi_eigenvalues_match_numpy(orc):
    rng = np.random.default_rng(11)
    for n in (2, 5, 9):
        G = rng.normal(size=(n, n))
        H = G + G.T
        S, W = orc.eig(H)
        np.testing.assert_allclose(np.sort(S), np.linalg.eigvalsh(H), atol=1e-12)
        np.testing.assert_allclose(W @ np.diag(S) @ W.T, H, atol=1e-12)
        np.testing.assert_allclose(W.T @ W, np.eye(n), atol=1e-13)
