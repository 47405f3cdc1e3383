"""The paper's partitioned solve of one periodic tridiagonal system (Sec.
"Linear Solver", eq:BlockSchurSystem and the three problems eq:LocalTriSystem,
eq:SchurSystem, eq:SchurCorrection), plain numpy in FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle): it states the paper's
subdomain algorithm so that tests can pin it to the plain cyclic solve; the
HIP library neither imports nor mirrors it.

Notation as in the paper: row i reads  c_i x_{i-1} + a_i x_i + b_i x_{i+1} = f_i
with indices taken mod N (c_0 and b_{N-1} are the periodic corners).  The
line is cut into P contiguous subdomains; the first unknown of subdomain p is
its interface unknown y_p, the others are its interior unknowns x_p.
Reordering interior unknowns first and interface unknowns last gives the
block system [[B, E], [F, C]] [x; y] = [f; g] with B block diagonal (one
non-periodic tridiagonal block B_p per subdomain).  Its Schur complement
S = C - F B^{-1} E couples each y_p only to y_{p-1} and y_{p+1}, so the
solve is: local solves B_p f*_p = f_p, the P x P system S y = g - F f*, and
the local corrections x_p = f*_p - B_p^{-1} E_p y.
"""
from __future__ import annotations

import numpy as np


def thomas(c, a, b, f):
    """Non-periodic tridiagonal solve (Thomas's algorithm): c[i] x[i-1] +
    a[i] x[i] + b[i] x[i+1] = f[i], with c[0] and b[-1] unused."""
    n = len(a)
    cp = np.zeros(n)
    fp = np.zeros(n)
    cp[0] = b[0] / a[0] if n > 1 else 0.0
    fp[0] = f[0] / a[0]
    for i in range(1, n):
        den = a[i] - c[i] * cp[i - 1]
        cp[i] = b[i] / den if i < n - 1 else 0.0
        fp[i] = (f[i] - c[i] * fp[i - 1]) / den
    x = np.zeros(n)
    x[-1] = fp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = fp[i] - cp[i] * x[i + 1]
    return x


def bounds(N: int, P: int):
    """Start index of each of the P subdomains (sizes differ by at most 1),
    and N at the end."""
    return [(p * N) // P for p in range(P)] + [N]


def _local(c, a, b, f, st):
    """eq:LocalTriSystem per subdomain, and the two columns of B_p^{-1} E_p:
    the interior of subdomain p meets y_p through its first row (coefficient
    c) and y_{p+1}, the first unknown of the next subdomain, through its last
    row (coefficient b)."""
    fs, L, R = [], [], []
    for p in range(len(st) - 1):
        I = np.arange(st[p] + 1, st[p + 1])
        m = len(I)
        fs.append(thomas(c[I], a[I], b[I], f[I]))
        e = np.zeros(m)
        e[0] = c[I[0]]
        L.append(thomas(c[I], a[I], b[I], e))
        e = np.zeros(m)
        e[-1] = b[I[-1]]
        R.append(thomas(c[I], a[I], b[I], e))
    return fs, L, R


def _schur(c, a, b, f, st, fs, L, R):
    """eq:SchurSystem: row p is the equation of y_p, whose neighbours are the
    last interior unknown of subdomain p-1 and the first of subdomain p;
    substituting x = f* - L y_left - R y_right gives S and the right side
    g - F f*.  Indices are mod P (P = 1, 2 fold neighbours together)."""
    P = len(st) - 1
    S = np.zeros((P, P))
    rhs = np.zeros(P)
    for p in range(P):
        s = st[p]
        q = (p - 1) % P
        S[p, p] += a[s]
        # c_s x_{s-1},  x_{s-1} = f*_q[-1] - L_q[-1] y_q - R_q[-1] y_p
        S[p, q] -= c[s] * L[q][-1]
        S[p, p] -= c[s] * R[q][-1]
        # b_s x_{s+1},  x_{s+1} = f*_p[0] - L_p[0] y_p - R_p[0] y_{p+1}
        S[p, p] -= b[s] * L[p][0]
        S[p, (p + 1) % P] -= b[s] * R[p][0]
        rhs[p] = f[s] - c[s] * fs[q][-1] - b[s] * fs[p][0]
    return S, rhs


def _check(N, P):
    st = bounds(N, P)
    if P < 1 or min(st[p + 1] - st[p] for p in range(P)) < 2:
        raise ValueError("every subdomain needs two or more unknowns")
    return st


def partitioned_cyclic_solve(c, a, b, f, P: int):
    """Solve the periodic system by the paper's P-subdomain Schur-complement
    procedure.  Every subdomain needs at least two unknowns (its interface
    unknown and at least one interior one)."""
    c, a, b, f = (np.asarray(v, dtype=np.float64) for v in (c, a, b, f))
    st = _check(len(a), P)
    fs, L, R = _local(c, a, b, f, st)
    S, rhs = _schur(c, a, b, f, st, fs, L, R)
    y = np.linalg.solve(S, rhs)
    # eq:SchurCorrection
    x = np.zeros(len(a))
    for p in range(P):
        x[st[p]] = y[p]
        x[st[p] + 1:st[p + 1]] = fs[p] - L[p] * y[p] - R[p] * y[(p + 1) % P]
    return x


def schur_matrix(c, a, b, P: int):
    """S = C - F B^{-1} E alone, assembled as in the solve."""
    c, a, b = (np.asarray(v, dtype=np.float64) for v in (c, a, b))
    st = _check(len(a), P)
    zero = np.zeros(len(a))
    fs, L, R = _local(c, a, b, zero, st)
    return _schur(c, a, b, zero, st, fs, L, R)[0]
