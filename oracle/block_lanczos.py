"""Oracle: block Lanczos with full reorthogonalisation (plain FP64 / complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names "(block) Lanczos" as its eigen-solver for the states near the
gap (Sec. III-A, item 1).  Block Lanczos carries a block of b orthonormal
vectors instead of one, so an eigenvalue of multiplicity up to b (the
degenerate states of a symmetric crystal, Kramers pairs with spin-orbit)
appears with its full multiplicity among the Ritz values, and a start block
can hold several approximate eigenvectors at once (warm starts inside the
self-consistent loop).

With Q_1 R_0 = X0 (QR), Q_0 = 0 and B_1 = R_0, for j = 1..m:

    W   = H Q_j - Q_{j-1} B_j^H
    A_j = Q_j^H W
    W  -= Q_j A_j
    [full reorthogonalisation: twice { W -= Q (Q^H W) } over Q_1..Q_j]
    Q_{j+1} B_{j+1} = W                      (QR)

so that H [Q_1..Q_m] = [Q_1..Q_m] T_m + Q_{m+1} B_{m+1} E_m^H with T_m the
Hermitian block-tridiagonal matrix of the A_j (diagonal) and B_j
(sub-diagonal).  Rayleigh-Ritz: T_m S = S Theta; Ritz vectors Y = Q S;
residuals |H y - theta y| with an explicit product.  Written from these
definitions; numpy's eigh serves as the dense eigensolver step.

Deflation.  When W loses rank (an eigenspace of multiplicity above b, or an
exactly invariant start block), the QR step is Gram-Schmidt column by column
(twice), and a column whose remainder is at most defl_tol |H| (|H| the
largest entry of the A_j and B_j so far; for the start block, its largest
column norm) is deflated:
its row of B_{j+1} is zero and its new basis vector is a pseudo-random vector
orthogonalised against every basis vector so far.  The pseudo-random values
come from the SplitMix64 generator (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) at counter
((j b + i) << 32) + e for element e of column i at step j; the library
implements the same generator, so both sides deflate into the same vectors.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output for the uint64 counters x (array)."""
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def deflation_vector(step, col, b, n, cplx):
    """Replacement vector of column col at block step step: uniform [-1, 1)
    entries 2 (s >> 11) 2^-53 - 1 of s = splitmix64(counter); complex vectors
    take their real and imaginary parts from elements 2e and 2e + 1."""
    ne = 2 * n if cplx else n
    base = np.uint64((step * b + col) << 32)
    with np.errstate(over="ignore"):
        s = splitmix64(base + np.arange(ne, dtype=np.uint64))
    u = (s >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0
    return u[0::2] + 1j * u[1::2] if cplx else u


def qr_deflate(W, Qall, step, hnorm, defl_tol, Qorth=None):
    """W = Qn Bn by column-wise Gram-Schmidt: each column twice against the
    basis so far and the new columns before it (the coefficients on the new
    columns form Bn; those on the old basis are rounding-level, since W is
    already orthogonal to it, and are dropped).  Columns with remainder
    <= defl_tol * hnorm are replaced as described in the module docstring."""
    n, b = W.shape
    cplx = np.iscomplexobj(W)
    Qn = np.zeros_like(W)
    Bn = np.zeros((b, b), dtype=W.dtype)
    Qorth = Qall if Qorth is None else Qorth     # without reorthogonalisation: none
    k0 = Qorth.shape[1]
    for i in range(b):
        w = W[:, i].copy()
        basis = np.hstack([Qorth, Qn[:, :i]])
        for _ in range(2):
            c = basis.conj().T @ w
            w = w - basis @ c
            Bn[:i, i] += c[k0:]
        nr = np.linalg.norm(w)
        if nr > defl_tol * hnorm:
            Bn[i, i] = nr
            Qn[:, i] = w / nr
            continue
        # deflated: B's entries of this column stay as accumulated (the
        # remainder w is dropped), the basis vector is a fresh direction
        v = deflation_vector(step, i, b, n, cplx).astype(W.dtype)
        basis = np.hstack([Qall, Qn[:, :i]])
        for _ in range(2):
            v = v - basis @ (basis.conj().T @ v)
        Qn[:, i] = v / np.linalg.norm(v)
    return Qn, Bn


def block_lanczos(matvec, X0, m, reorth=True, defl_tol=1e-12):
    """m block steps from the start block X0 [n, b].  matvec(X) returns H X
    for a block.  Returns dict(Q [n, (m+1) b] (the last block is Q_{m+1}),
    A [m][b, b], B [m+1][b, b] (B[0] = R_0, B[j] couples blocks j-1 and j),
    T [m b, m b], deflated = number of deflated columns)."""
    X0 = np.asarray(X0)
    n, b = X0.shape
    dt = np.result_type(X0.dtype, np.float64)
    X0 = X0.astype(dt)
    Q1, R0 = qr_deflate(X0, np.zeros((n, 0), dtype=dt), 0, np.linalg.norm(X0, axis=0).max(), defl_tol)
    Qs = [Q1]
    As, Bs = [], [R0]
    Qprev = np.zeros((n, b), dtype=dt)
    Bj = np.zeros((b, b), dtype=dt)
    hnorm = 0.0
    for j in range(m):
        Qj = Qs[j]
        W = matvec(Qj) - Qprev @ Bj.conj().T
        Aj = Qj.conj().T @ W
        W = W - Qj @ Aj
        Qall = np.hstack(Qs)
        if reorth:
            for _ in range(2):
                W = W - Qall @ (Qall.conj().T @ W)
        hnorm = max(hnorm, np.abs(Aj).max(), np.abs(Bj).max())
        Qn, Bn = qr_deflate(W, Qall, j + 1, hnorm, defl_tol, None if reorth else Qall[:, :0])
        As.append(0.5 * (Aj + Aj.conj().T))
        Bs.append(Bn)
        Qs.append(Qn)
        Qprev, Bj = Qj, Bn
    T = np.zeros((m * b, m * b), dtype=dt)
    for j in range(m):
        T[j * b:(j + 1) * b, j * b:(j + 1) * b] = As[j]
        if j + 1 < m:
            T[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = Bs[j + 1]
            T[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = Bs[j + 1].conj().T
    return dict(Q=np.hstack(Qs), A=As, B=Bs, T=T)


def block_lanczos_eigs(matvec, X0, m, sigma, k, res_tol=1e-4, reorth=True, defl_tol=1e-12):
    """Ritz pairs of m block steps; the k converged Ritz values nearest sigma
    (each copy of a repeated eigenvalue is its own Ritz pair).  Returns
    dict(theta [k] ascending, res [k], Y [n, k], theta_all, res_all)."""
    r = block_lanczos(matvec, X0, m, reorth, defl_tol)
    nb = r["T"].shape[0]
    th, S = np.linalg.eigh(r["T"])
    Y = r["Q"][:, :nb] @ S
    R = matvec(Y) - Y * th[None, :]
    res = np.linalg.norm(R, axis=0)
    ok = np.flatnonzero(res <= res_tol)
    order = ok[np.lexsort((th[ok], np.abs(th[ok] - sigma)))][:k]
    sel = np.sort(order)
    sel = sel[np.argsort(th[sel], kind="stable")]
    return dict(theta=th[sel], res=res[sel], Y=Y[:, sel], theta_all=th, res_all=res, steps=m)
