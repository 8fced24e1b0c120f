"""FMM translation operators for the 2D Helmholtz kernel, as plain sums.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation (points are complex numbers z = x + i y):
  O_n(z) = H_n(omega|z|) e^{i n arg z}   outgoing ("H-expansion") basis,
  I_n(z) = J_n(omega|z|) e^{i n arg z}   incoming basis,
  L_n(z) = J_n(omega|z|) e^{-i n arg z} = (-1)^n I_{-n}(z), the paper's
           local ("J-expansion") basis (Sec. 2.1, eq. (jexp); Sec. 7).
A multipole about m is  phi(x) = sum_k a_k O_k(x - m)  (Sec. 7.1);
a local about c is      psi(x) = sum_l g_l L_l(x - c)   (Sec. 7).

The operators follow from Graf's addition theorem (Sec. 2.1) in the forms
  O_n(x + y) = sum_k O_{n-k}(x) I_k(y),  |y| < |x|,
  I_n(x + y) = sum_k I_{n-k}(x) I_k(y):
  P2M  a_k  = q L_k(s - m)                        (Sec. 7.1, a_k formula)
  M2M  a_n  = sum_k a'_k I_{k-n}(m - m')          (child m' -> parent m; Stage 2)
  M2L  g_l  = (-1)^l sum_k a_k O_{k+l}(c - m)     (Stage 4; also M2QBXL, Stage 5)
  L2L  g'_l = sum_k g_k I_{l-k}(c - c')           (Stage 7; also L2QBXL, Stage 8)
  P2L  g_l  = q O_l(s - c)                        (Sec. 2.1 eq. (graf-coefficient);
                                                   P2QBXL Stage 3 and X-list Stage 6)
Dipole sources (double layer, strength q, unit normal nu = n_x + i n_y):
  P2M  a_k += q (omega/2) (conj(nu) L_{k-1}(s-m) - nu L_{k+1}(s-m))
  P2L  g_l += q (omega/2) (nu O_{l-1}(s-c) - conj(nu) O_{l+1}(s-c))
"""
from __future__ import annotations

import numpy as np

from . import besselj_seq, hankel1_seq


def _signed_range(nmin, nmax):
    return np.arange(nmin, nmax + 1)


def outgoing(omega, z, nmin, nmax):
    """O_n(z) for n = nmin..nmax."""
    z = complex(z)
    N = max(abs(nmin), abs(nmax))
    h = hankel1_seq(omega * abs(z), N)
    n = _signed_range(nmin, nmax)
    hn = h[np.abs(n)] * np.where((n < 0) & (np.abs(n) % 2 == 1), -1.0, 1.0)
    return hn * np.exp(1j * n * np.angle(z))


def incoming(omega, z, nmin, nmax):
    """I_n(z) for n = nmin..nmax."""
    z = complex(z)
    N = max(abs(nmin), abs(nmax))
    j = besselj_seq(omega * abs(z), N)
    n = _signed_range(nmin, nmax)
    jn = j[np.abs(n)] * np.where((n < 0) & (np.abs(n) % 2 == 1), -1.0, 1.0)
    return jn * np.exp(1j * n * np.angle(z))


def local_basis(omega, z, P):
    """L_l(z), l = -P..P."""
    z = complex(z)
    j = besselj_seq(omega * abs(z), P)
    n = _signed_range(-P, P)
    jn = j[np.abs(n)] * np.where((n < 0) & (np.abs(n) % 2 == 1), -1.0, 1.0)
    return jn * np.exp(-1j * n * np.angle(z))


def p2m(omega, m, s, qs, qd, nu, P):
    """Multipole coefficients a_k, k = -P..P, about m of charges qs and dipoles
    (qd, nu) at points s (arrays)."""
    a = np.zeros(2 * P + 1, dtype=np.complex128)
    for sj, qsj, qdj, nuj in zip(np.atleast_1d(s), np.atleast_1d(qs), np.atleast_1d(qd),
                                 np.atleast_1d(nu)):
        Lk = local_basis(omega, sj - m, P + 1)          # index k + P + 1
        a += qsj * Lk[1:-1]
        a += qdj * 0.5 * omega * (np.conj(nuj) * Lk[:-2] - nuj * Lk[2:])
    return a


def m2m(omega, a_child, m_child, m_parent, P_parent):
    Pc = (a_child.size - 1) // 2
    k = _signed_range(-Pc, Pc)
    Ivals = incoming(omega, m_parent - m_child, -(Pc + P_parent), Pc + P_parent)
    off = Pc + P_parent
    out = np.zeros(2 * P_parent + 1, dtype=np.complex128)
    for i, n in enumerate(_signed_range(-P_parent, P_parent)):
        out[i] = np.sum(a_child * Ivals[k - n + off])
    return out


def m2l(omega, a, m, c, P_local):
    P = (a.size - 1) // 2
    k = _signed_range(-P, P)
    Ovals = outgoing(omega, c - m, -(P + P_local), P + P_local)
    off = P + P_local
    out = np.zeros(2 * P_local + 1, dtype=np.complex128)
    for i, l in enumerate(_signed_range(-P_local, P_local)):
        out[i] = (-1.0) ** (l % 2) * np.sum(a * Ovals[k + l + off])
    return out


def l2l(omega, g, c, c_new, P_new):
    P = (g.size - 1) // 2
    k = _signed_range(-P, P)
    Ivals = incoming(omega, c - c_new, -(P + P_new), P + P_new)
    off = P + P_new
    out = np.zeros(2 * P_new + 1, dtype=np.complex128)
    for i, l in enumerate(_signed_range(-P_new, P_new)):
        out[i] = np.sum(g * Ivals[l - k + off])
    return out


def p2l(omega, c, s, qs, qd, nu, P):
    g = np.zeros(2 * P + 1, dtype=np.complex128)
    for sj, qsj, qdj, nuj in zip(np.atleast_1d(s), np.atleast_1d(qs), np.atleast_1d(qd),
                                 np.atleast_1d(nu)):
        O = outgoing(omega, sj - c, -(P + 1), P + 1)    # index l + P + 1
        g += qsj * O[1:-1]
        g += qdj * 0.5 * omega * (nuj * O[:-2] - np.conj(nuj) * O[2:])
    return g


def m2p(omega, a, m, x):
    P = (a.size - 1) // 2
    return np.sum(a * outgoing(omega, x - m, -P, P))


def l2p(omega, g, c, x):
    P = (g.size - 1) // 2
    return np.sum(g * local_basis(omega, x - c, P))
