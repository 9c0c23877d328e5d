"""Pins of the oracle's frozen-Q backward: central finite differences of the
bilinear surrogate C = Q Q^T A B in FP64 (exact up to rounding because the
map is bilinear in (A, B) once Q is fixed)."""

import numpy as np

import synth
from oracle import lramm as L
from oracle.qr import householder_qr


def _frozen_q(A, l, seed):
    om = synth.omega(A.shape[1], l, seed).astype(np.float64)
    return householder_qr(A @ om)[0]


def test_directional_fd_256():
    m = k = n = 256
    A, _ = synth.lowrank(m, k, synth.spectrum("exp", 256, 32.0), 0)
    A = A.astype(np.float64)
    B = synth.gaussian(k, n, 100).astype(np.float64)
    Q = _frozen_q(A, 74, 1)
    rng = np.random.default_rng(2)
    dC = rng.standard_normal((m, n))
    dA, dB = L.lramm_backward(Q, A, B, dC)
    h = 1e-6
    for _ in range(4):
        EA = rng.standard_normal((m, k))
        EB = rng.standard_normal((k, n))
        fa = (np.sum(dC * L.surrogate(Q, A + h * EA, B)) - np.sum(dC * L.surrogate(Q, A - h * EA, B))) / (2 * h)
        fb = (np.sum(dC * L.surrogate(Q, A, B + h * EB)) - np.sum(dC * L.surrogate(Q, A, B - h * EB))) / (2 * h)
        assert abs(fa - np.sum(dA * EA)) <= 1e-9 * abs(fa) + 1e-9
        assert abs(fb - np.sum(dB * EB)) <= 1e-9 * abs(fb) + 1e-9


def test_entrywise_fd_tiny():
    rng = np.random.default_rng(3)
    m, k, n = 6, 5, 4
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    Q = householder_qr(rng.standard_normal((m, 3)))[0]
    dC = rng.standard_normal((m, n))
    dA, dB = L.lramm_backward(Q, A, B, dC)
    h = 1e-5
    for i in range(m):
        for j in range(k):
            E = np.zeros_like(A)
            E[i, j] = h
            fd = (np.sum(dC * L.surrogate(Q, A + E, B)) - np.sum(dC * L.surrogate(Q, A - E, B))) / (2 * h)
            assert abs(fd - dA[i, j]) <= 1e-9
    for i in range(k):
        for j in range(n):
            E = np.zeros_like(B)
            E[i, j] = h
            fd = (np.sum(dC * L.surrogate(Q, A, B + E)) - np.sum(dC * L.surrogate(Q, A, B - E))) / (2 * h)
            assert abs(fd - dB[i, j]) <= 1e-9
