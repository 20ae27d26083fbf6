"""Oracle: Lanczos eigensolver for the states nearest a target energy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Schrodinger step solves the tight-binding eigenproblem with an
iterative (block) Lanczos solver (Sec. III-A, item 1), and its benchmark unit
is a fixed number of Lanczos iterations (Sec. II-B, Figs. 2-3).  The paper
gives no algorithm listing, so this is the textbook symmetric Lanczos
recurrence in FP64 with full reorthogonalisation by classical Gram-Schmidt
applied twice (CGS2), followed by Rayleigh-Ritz on the tridiagonal matrix:

    w = H v_j - beta_j v_{j-1};  alpha_j = Re(v_j^H w);  w -= alpha_j v_j
    twice: c = V_j^H w;  w -= V_j c        (alpha_j is not corrected)
    beta_{j+1} = ||w||;  v_{j+1} = w / beta_{j+1}

Breakdown: beta_{j+1} <= 1e-12 * max|T| stops the recurrence with j steps.

Result contract (the paper is silent on interior targets and multiplicity):
Ritz pairs nearest sigma are candidates; a candidate is converged when its
explicit FP64 residual ||H y - theta y|| (||y|| = 1) is <= res_tol; converged
values closer than merge_tol are one eigenvalue (copy count reported); the k
distinct converged values nearest sigma are returned ascending, each with its
Rayleigh-quotient refinement y^H H y.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos(hx, v0, m, reorth=True, breakdown_rel=1e-12):
    """Run m Lanczos steps.  Returns (alpha[m'], beta[m'] (beta[j] couples
    steps j and j+1; beta[m'-1] is the residual norm), V[m', dim])."""
    v0 = np.asarray(v0)
    dim = v0.shape[0]
    V = np.zeros((m, dim), dtype=v0.dtype)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    V[0] = v0 / np.linalg.norm(v0)
    b_prev = 0.0
    tmax = 0.0
    steps = 0
    for j in range(m):
        w = hx(V[j])
        if j > 0:
            w = w - b_prev * V[j - 1]
        a = float(np.real(np.vdot(V[j], w)))
        w = w - a * V[j]
        if reorth:
            for _ in range(2):
                c = V[: j + 1].conj() @ w
                w = w - V[: j + 1].T @ c
        b = float(np.linalg.norm(w))
        alpha[j] = a
        beta[j] = b
        steps = j + 1
        tmax = max(tmax, abs(a), b)
        if b <= breakdown_rel * tmax:
            break
        if j + 1 < m:
            V[j + 1] = w / b
        b_prev = b
    return alpha[:steps], beta[:steps], V[:steps]


def tridiag_eig(alpha, beta):
    """Eigenvalues ascending and eigenvectors of T (FP64, LAPACK stemr; the
    implicit-QL driver stev when stemr reports non-convergence, which it does
    on the tight clusters that ghost copies of a long unreorthogonalised run
    form)."""
    off = beta[: len(alpha) - 1]
    try:
        return eigh_tridiagonal(alpha, off)
    except np.linalg.LinAlgError:
        return eigh_tridiagonal(alpha, off, lapack_driver="stev")


def select_converged(theta, res, refined, sigma, k, merge_tol=1e-6, res_tol=1e-4):
    """Distinct converged eigenvalues nearest sigma.

    A candidate's value is its Rayleigh quotient with the FP64 H (``refined``;
    for a converged pair it is within res^2 / gap of the eigenvalue, while
    the raw Ritz value of a reduced-precision recurrence can be off by more
    than merge_tol).  Converged candidates are clustered: sorted by value, a
    gap larger than merge_tol starts a new cluster.  A cluster's
    representative is its member with the smallest residual.  The k clusters
    nearest sigma (ties: smaller value) are returned ascending as dict
    arrays."""
    theta = np.asarray(theta)
    val = np.asarray(refined)
    conv = np.flatnonzero(np.asarray(res) <= res_tol)
    if conv.size == 0:
        return dict(theta=np.zeros(0), refined=np.zeros(0), res=np.zeros(0), copies=np.zeros(0, int))
    o = conv[np.argsort(val[conv], kind="stable")]
    clusters = [[o[0]]]
    for a, b in zip(o[:-1], o[1:]):
        if val[b] - val[a] > merge_tol:
            clusters.append([b])
        else:
            clusters[-1].append(b)
    reps = []
    for cl in clusters:
        r = min(cl, key=lambda i: (res[i], i))
        reps.append((r, len(cl)))
    reps.sort(key=lambda rc: (abs(val[rc[0]] - sigma), val[rc[0]]))
    reps = reps[:k]
    reps.sort(key=lambda rc: val[rc[0]])
    idx = np.array([r for r, _ in reps], dtype=int)
    return dict(theta=theta[idx], refined=np.asarray(refined)[idx], res=np.asarray(res)[idx],
                copies=np.array([c for _, c in reps], dtype=int), index=idx)


def n_candidates(k, m):
    """Candidate Ritz pairs examined for a request of k values."""
    return min(m, max(4 * k, k + 16))


def lanczos_eigs(hx, v0, m, sigma, k, reorth=True, res_tol=1e-4, merge_tol=1e-6, hx_ref=None):
    """Full driver: Lanczos, tridiagonal eigensolve, candidates nearest sigma,
    Ritz vectors, explicit residuals and Rayleigh-quotient refinement with
    ``hx_ref`` (defaults to ``hx``)."""
    hx_ref = hx if hx_ref is None else hx_ref
    alpha, beta, V = lanczos(hx, v0, m, reorth=reorth)
    th, S = tridiag_eig(alpha, beta)
    nc = n_candidates(k, len(alpha))
    cand = np.argsort(np.abs(th - sigma), kind="stable")[:nc]
    theta = th[cand]
    res = np.zeros(nc)
    ref = np.zeros(nc)
    Y = S[:, cand].T @ V
    for c in range(nc):
        y = Y[c]
        nrm2 = float(np.real(np.vdot(y, y)))
        hy = hx_ref(y)
        ref[c] = float(np.real(np.vdot(y, hy))) / nrm2
        res[c] = float(np.linalg.norm(hy - theta[c] * y)) / np.sqrt(nrm2)
    sel = select_converged(theta, res, ref, sigma, k, merge_tol, res_tol)
    sel.update(alpha=alpha, beta=beta, ritz_all=th, cand_theta=theta, cand_res=res,
               cand_refined=ref, steps=len(alpha))
    return sel
