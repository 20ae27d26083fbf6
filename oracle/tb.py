"""Oracle: empirical tight-binding Hamiltonian on a diamond lattice.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's electronic structure is the empirical sp3s* / sp3d5s*
nearest-neighbour tight-binding model with strain (Abstract; Sec. I, "Need
for Atomistic Modeling" and "Multi-Million Atom Simulations"), solved on
finite k-points (Sec. III-A, item 1).  It prints no formula, so this module
writes the textbook model out from its definitions:

* neighbours: atoms at the nearest-neighbour distance sqrt(3)*a/4, found by
  searching every displacement of that length (periodic axes wrap);
* two-centre hopping blocks (Slater & Koster, Phys. Rev. 94, 1498 (1954)):
  built by rotating the bond-along-z block with numerically fitted real
  spherical-harmonic representation matrices, B(d) = D(R) B_z D(R)^T with
  R z = d;
* on-site block: orbital energies, per-atom potential, spin-orbit
  lambda L.S on the p shell (lambda = 2 Delta_so / 3), and a +E_pass shift of
  each dangling bond's sp3 hybrid;
* Bloch phase exp(2 pi i k_frac . w) for a bond that wraps by w boxes.

Rows are atom-major, orbital-minor, spin-major within an atom:
row = atom * n_o + spin * n_base + orbital.

Orbital order: sp3s* = [s, px, py, pz, s*];
sp3d5s* = [s, px, py, pz, dxy, dyz, dzx, dx2-y2, d3z2-r2, s*].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MODEL_SP3S = 0
MODEL_SP3D5S = 1

# slot directions for sublattice A (a/4 units); sublattice B uses -d
SLOT_DIRS = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.int64)

# indices into the 14 two-centre integrals
SS, SSTSST, SSST, SP, SSTP, SD, SSTD, PPS, PPP, PDS, PDP, DDS, DDP, DDD = range(14)


def sublattice(pos_q):
    """0 for sublattice A (x+y+z = 0 mod 4), 1 for B (= 3 mod 4)."""
    r = np.asarray(pos_q, dtype=np.int64).sum(axis=1) % 4
    if np.any((r != 0) & (r != 3)):
        raise ValueError("positions are not on the diamond lattice")
    return (r == 3).astype(np.int64)


def find_neighbours(pos_q, box_q, periodic):
    """Nearest-neighbour table by search over all displacements of length
    sqrt(3) a/4 (the eight vectors (+-1,+-1,+-1) in a/4 units).

    Returns nbr [N,4] (int32, -1 = dangling) and wrap [N,4,3] (int8): the
    neighbour of atom i in slot b sits at pos[nbr] + wrap*box = pos[i] + d,
    d = +SLOT_DIRS[b] on sublattice A and -SLOT_DIRS[b] on B."""
    pos = np.asarray(pos_q, dtype=np.int64)
    box = np.asarray(box_q, dtype=np.int64)
    per = np.asarray(periodic, dtype=bool)
    N = pos.shape[0]
    sub = sublattice(pos)
    span = box + 8
    def key(p):
        q = p + 4
        return (q[:, 2] * span[1] + q[:, 1]) * span[0] + q[:, 0]
    keys = key(pos)
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    if np.any(skeys[1:] == skeys[:-1]):
        raise ValueError("duplicate atom positions")
    nbr = np.full((N, 4), -1, dtype=np.int32)
    wrap = np.zeros((N, 4, 3), dtype=np.int8)
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                d = np.array([sx, sy, sz], dtype=np.int64)
                t = pos + d
                w = np.zeros_like(t)
                for ax in range(3):
                    if per[ax]:
                        w[:, ax] = np.floor_divide(t[:, ax], box[ax])
                        t[:, ax] -= w[:, ax] * box[ax]
                k = key(t)
                idx = np.minimum(np.searchsorted(skeys, k), N - 1)
                hit = np.flatnonzero(skeys[idx] == k)
                if hit.size == 0:
                    continue
                # the signed slot direction: +d on A, -d on B
                slot_a = np.flatnonzero((SLOT_DIRS == d).all(axis=1))
                slot_b = np.flatnonzero((SLOT_DIRS == -d).all(axis=1))
                for s_val, slot in ((0, slot_a), (1, slot_b)):
                    ii = hit[sub[hit] == s_val]
                    if ii.size == 0:
                        continue
                    if slot.size != 1:
                        raise ValueError("neighbour in a non-bond direction")
                    b = int(slot[0])
                    if np.any(nbr[ii, b] != -1):
                        raise ValueError(f"two neighbours in slot {b}")
                    nbr[ii, b] = order[idx[ii]]
                    wrap[ii, b] = w[ii]
    return nbr, wrap


def brute_force_neighbours(pos_q, box_q, periodic):
    """O(N^2) check: all pairs at squared distance 3 under the minimum image."""
    pos = np.asarray(pos_q, dtype=np.int64)
    box = np.asarray(box_q, dtype=np.int64)
    out = []
    for i in range(pos.shape[0]):
        d = pos - pos[i]
        for ax in range(3):
            if periodic[ax]:
                d[:, ax] -= box[ax] * np.round(d[:, ax] / box[ax]).astype(np.int64)
        r2 = (d * d).sum(axis=1)
        out.append(set(np.flatnonzero(r2 == 3).tolist()))
    return out


# ---------------------------------------------------------------------------
# Slater-Koster blocks by rotation
# ---------------------------------------------------------------------------

def _real_harmonics(l, r):
    """Real harmonics (common normalisation) evaluated at unit vectors r."""
    x, y, z = r[:, 0], r[:, 1], r[:, 2]
    if l == 1:
        return np.stack([x, y, z], axis=1)
    s3 = np.sqrt(3.0)
    return np.stack([s3 * x * y, s3 * y * z, s3 * z * x,
                     0.5 * s3 * (x * x - y * y), z * z - 0.5 * (x * x + y * y)], axis=1)


def rep_matrix(l, R, rng=None):
    """Representation matrix D with f_a(R^T r) = sum_b D[b, a] f_b(r), fitted
    by least squares at random points on the unit sphere."""
    rng = np.random.default_rng(12345) if rng is None else rng
    pts = rng.standard_normal((64, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    F = _real_harmonics(l, pts)
    G = _real_harmonics(l, pts @ R)          # rows: f(R^T r) with r as row vectors
    D, *_ = np.linalg.lstsq(F, G, rcond=None)
    return D


def rotation_to(d):
    """A proper rotation R with R e_z = d (d unit)."""
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = a - np.dot(a, d) * d
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return np.stack([e1, e2, d], axis=1)


def n_base_orbitals(model):
    return 5 if model == MODEL_SP3S else 10


def bond_block_z(model, V):
    """Hopping block <i a|H|j b> for j displaced from i along +z."""
    nb = n_base_orbitals(model)
    B = np.zeros((nb, nb))
    s, px, py, pz = 0, 1, 2, 3
    st = nb - 1
    B[s, s] = V[SS]
    B[st, st] = V[SSTSST]
    B[s, st] = B[st, s] = V[SSST]
    B[s, pz], B[pz, s] = V[SP], -V[SP]
    B[st, pz], B[pz, st] = V[SSTP], -V[SSTP]
    B[px, px] = B[py, py] = V[PPP]
    B[pz, pz] = V[PPS]
    if model == MODEL_SP3D5S:
        dxy, dyz, dzx, dx2, dz2 = 4, 5, 6, 7, 8
        B[s, dz2] = B[dz2, s] = V[SD]
        B[st, dz2] = B[dz2, st] = V[SSTD]
        B[pz, dz2], B[dz2, pz] = V[PDS], -V[PDS]
        B[px, dzx], B[dzx, px] = V[PDP], -V[PDP]
        B[py, dyz], B[dyz, py] = V[PDP], -V[PDP]
        B[dz2, dz2] = V[DDS]
        B[dzx, dzx] = B[dyz, dyz] = V[DDP]
        B[dxy, dxy] = B[dx2, dx2] = V[DDD]
    return B


def orbital_rep(model, R):
    """Block-diagonal rotation of the orbital basis: 1 (s) + D1 (p) [+ D2 (d)] + 1 (s*)."""
    nb = n_base_orbitals(model)
    D = np.zeros((nb, nb))
    D[0, 0] = 1.0
    D[nb - 1, nb - 1] = 1.0
    D[1:4, 1:4] = rep_matrix(1, R)
    if model == MODEL_SP3D5S:
        D[4:9, 4:9] = rep_matrix(2, R)
    return D


def sk_block(model, V, d):
    """Two-centre block for the bond direction d (any length)."""
    R = rotation_to(d)
    D = orbital_rep(model, R)
    return D @ bond_block_z(model, V) @ D.T


# ---------------------------------------------------------------------------
# on-site
# ---------------------------------------------------------------------------

def angular_momentum_p():
    """L_k on (px, py, pz): (L_k)_{ab} = -i eps_{kab}."""
    L = np.zeros((3, 3, 3), dtype=complex)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    for k in range(3):
        L[k] = -1j * eps[k]
    return L


def spin_orbit_block(model, delta):
    """lambda sum_k S_k (x) L_k on the p shell in the spin-major basis
    [orbitals up, orbitals down], lambda = 2 Delta / 3, S = sigma / 2."""
    nb = n_base_orbitals(model)
    lam = 2.0 * delta / 3.0
    sig = [np.array([[0, 1], [1, 0]], dtype=complex),
           np.array([[0, -1j], [1j, 0]], dtype=complex),
           np.array([[1, 0], [0, -1]], dtype=complex)]
    L = angular_momentum_p()
    H = np.zeros((2 * nb, 2 * nb), dtype=complex)
    for k in range(3):
        Lfull = np.zeros((nb, nb), dtype=complex)
        Lfull[1:4, 1:4] = L[k]
        H += lam * np.kron(0.5 * sig[k], Lfull)
    return H


def hybrid_vector(model, d):
    """sp3 hybrid (s + d.p)/2 pointing along the bond direction d in {+-1}^3."""
    nb = n_base_orbitals(model)
    h = np.zeros(nb)
    h[0] = 0.5
    h[1:4] = 0.5 * np.asarray(d, dtype=np.float64)
    return h


def onsite_block(model, spin, E, U, so_delta, dangling_dirs, e_pass):
    """On-site block of one atom."""
    nb = n_base_orbitals(model)
    e = np.zeros(nb)
    e[0] = E[0]
    e[1:4] = E[1]
    if model == MODEL_SP3D5S:
        e[4:9] = E[2]
    e[nb - 1] = E[3]
    D = np.diag(e + U).astype(complex if spin else float)
    for d in dangling_dirs:
        h = hybrid_vector(model, d)
        D = D + e_pass * np.outer(h, h)
    if spin:
        D = np.kron(np.eye(2), D) + spin_orbit_block(model, so_delta)
    return D


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------

def build_blocks(prob):
    """All blocks of H: returns dict(nbr, wrap, onsite [N,n_o,n_o], bonds
    [N,4,n_o,n_o], n_o, complex).  Every bond block is computed from its own
    direction (no transpose shortcut), so Hermiticity is a check, not a
    construction."""
    par = prob.params
    model, spin = par["model"], par["spin"]
    nb = n_base_orbitals(model)
    n_o = nb * (2 if spin else 1)
    nbr, wrap = find_neighbours(prob.pos_q, prob.box_q, prob.periodic)
    N = nbr.shape[0]
    sub = sublattice(prob.pos_q)
    spc = np.asarray(prob.species, dtype=np.int64)
    ns = int(par["n_species"])
    kf = np.zeros(3) if prob.kfrac is None else np.asarray(prob.kfrac, dtype=np.float64)
    cplx = bool(spin) or bool(np.any(kf != 0))
    dt = complex if cplx else float
    U = np.zeros(N) if prob.onsite_pot is None else np.asarray(prob.onsite_pot, dtype=np.float64)

    # on-site: one block per (species, sublattice, dangling pattern)
    onsite = np.zeros((N, n_o, n_o), dtype=dt)
    dang_code = ((nbr < 0).astype(np.int64) * (1 << np.arange(4))).sum(axis=1)
    for s in range(ns):
        for sl in (0, 1):
            for code in range(16):
                sel = np.flatnonzero((spc == s) & (sub == sl) & (dang_code == code))
                if sel.size == 0:
                    continue
                sgn = 1 if sl == 0 else -1
                dirs = [sgn * SLOT_DIRS[b] for b in range(4) if code & (1 << b)]
                D = onsite_block(model, spin, par["onsite"][s], 0.0, par["so_delta"][s],
                                 dirs, par["passivation_eV"])
                onsite[sel] = D
    onsite += U[:, None, None] * np.eye(n_o)[None]

    # bonds: one base block per (species pair, signed direction), times the
    # strain factor of the bond's A atom and the Bloch phase of its wrap
    bonds = np.zeros((N, 4, n_o, n_o), dtype=dt)
    scale = np.ones((N, 4))
    if prob.bond_scale is not None:
        bs = np.asarray(prob.bond_scale, dtype=np.float64)
        for b in range(4):
            j = nbr[:, b]
            ok = j >= 0
            a_atom = np.where(sub == 0, np.arange(N), np.where(ok, j, 0))
            scale[:, b] = np.where(ok, bs[a_atom, b], 0.0)
    phase = np.exp(2j * np.pi * np.einsum("nbk,k->nb", wrap.astype(np.float64), kf))
    for b in range(4):
        j = nbr[:, b]
        for sl in (0, 1):
            sgn = 1 if sl == 0 else -1
            for sa in range(ns):
                for sb in range(ns):
                    sel = np.flatnonzero((j >= 0) & (sub == sl) & (spc == sa)
                                         & (spc[np.maximum(j, 0)] == sb))
                    if sel.size == 0:
                        continue
                    B = sk_block(model, par["sk"][sa][sb], sgn * SLOT_DIRS[b])
                    if spin:
                        B = np.kron(np.eye(2), B)
                    f = scale[sel, b]
                    if cplx:
                        f = f * phase[sel, b]
                    bonds[sel, b] = f[:, None, None] * B[None]
    return dict(nbr=nbr, wrap=wrap, onsite=onsite, bonds=bonds, n_o=n_o, complex=cplx)


def csr_hamiltonian(blk):
    """Scalar CSR matrix (FP64 / complex128) from the blocks."""
    nbr, onsite, bonds, n_o = blk["nbr"], blk["onsite"], blk["bonds"], blk["n_o"]
    N = nbr.shape[0]
    ar = np.arange(n_o)
    base = np.arange(N)[:, None, None] * n_o
    r = (base + ar[None, :, None]) + 0 * ar[None, None, :]
    parts_r, parts_c, parts_v = [r.ravel()], [(base + ar[None, None, :] + 0 * ar[None, :, None]).ravel()], [onsite.ravel()]
    for b in range(4):
        ok = nbr[:, b] >= 0
        jb = nbr[ok, b].astype(np.int64)[:, None, None] * n_o
        rb = (np.flatnonzero(ok)[:, None, None] * n_o + ar[None, :, None]) + 0 * ar[None, None, :]
        cb = (jb + ar[None, None, :]) + 0 * ar[None, :, None]
        parts_r.append(rb.ravel())
        parts_c.append(cb.ravel())
        parts_v.append(bonds[ok, b].ravel())
    H = sp.csr_matrix((np.concatenate(parts_v), (np.concatenate(parts_r), np.concatenate(parts_c))),
                      shape=(N * n_o, N * n_o))
    H.eliminate_zeros()
    return H


def hamiltonian(prob):
    """CSR H of a workloads.Problem."""
    return csr_hamiltonian(build_blocks(prob))


def hx(H, x):
    """y = H x (scalar CSR, FP64/complex128)."""
    return H @ x


# ---------------------------------------------------------------------------
# bulk Bloch Hamiltonian (two-atom primitive cell)
# ---------------------------------------------------------------------------

def bulk_hk(model, spin, E, V, so_delta, k_cart):
    """Bulk H(k) of the diamond primitive cell in the position gauge:
    H_AB(k) = sum_b B(d_b) exp(i k . d_b a/4), k in units of 1/(a/4)."""
    nb = n_base_orbitals(model)
    n_o = nb * (2 if spin else 1)
    D = onsite_block(model, spin, E, 0.0, so_delta, [], 0.0)
    HAB = np.zeros((n_o, n_o), dtype=complex)
    for b in range(4):
        B = sk_block(model, V, SLOT_DIRS[b])
        if spin:
            B = np.kron(np.eye(2), B)
        HAB += B * np.exp(1j * np.dot(k_cart, SLOT_DIRS[b]))
    H = np.zeros((2 * n_o, 2 * n_o), dtype=complex)
    H[:n_o, :n_o] = D
    H[n_o:, n_o:] = D
    H[:n_o, n_o:] = HAB
    H[n_o:, :n_o] = HAB.conj().T
    return H


def hx_rows(prob, atoms, x, nbr=None, wrap=None, absolute=False):
    """Rows of y = H x belonging to the given atoms, computed atom by atom
    from the definition (for spot checks at sizes where the full CSR matrix
    is too large).  Returns [len(atoms), n_o] (complex if H is complex).
    With absolute=True every block is replaced by its element-wise absolute
    value, giving (|H| x)_i: with x = |x| the scale of a row's rounding
    error bound."""
    par = prob.params
    model, spin = par["model"], par["spin"]
    nb = n_base_orbitals(model)
    n_o = nb * (2 if spin else 1)
    if nbr is None:
        nbr, wrap = find_neighbours(prob.pos_q, prob.box_q, prob.periodic)
    sub = sublattice(prob.pos_q)
    spc = np.asarray(prob.species, dtype=np.int64)
    kf = np.zeros(3) if prob.kfrac is None else np.asarray(prob.kfrac, dtype=np.float64)
    cplx = bool(spin) or bool(np.any(kf != 0))
    X = np.asarray(x).reshape(-1, n_o)
    out = np.zeros((len(atoms), n_o), dtype=complex if cplx else float)
    for r, i in enumerate(atoms):
        sgn = 1 if sub[i] == 0 else -1
        dirs = [sgn * SLOT_DIRS[b] for b in range(4) if nbr[i, b] < 0]
        U = 0.0 if prob.onsite_pot is None else prob.onsite_pot[i]
        D = onsite_block(model, spin, par["onsite"][spc[i]], U, par["so_delta"][spc[i]],
                         dirs, par["passivation_eV"])
        if absolute:
            D = np.abs(D)
        acc = D @ X[i]
        for b in range(4):
            j = nbr[i, b]
            if j < 0:
                continue
            B = sk_block(model, par["sk"][spc[i]][spc[j]], sgn * SLOT_DIRS[b])
            if prob.bond_scale is not None:
                B = B * prob.bond_scale[i if sub[i] == 0 else j, b]
            if spin:
                B = np.kron(np.eye(2), B)
            if cplx:
                B = B * np.exp(2j * np.pi * np.dot(kf, wrap[i, b]))
            if absolute:
                B = np.abs(B)
            acc = acc + B @ X[j]
        out[r] = acc
    return out
