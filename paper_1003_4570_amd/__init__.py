"""Python binding of libtbh.so: MI355X tight-binding H.x, Lanczos and
Schrodinger-Poisson.

Argument marshalling only: every step runs in the library's HIP kernels.
Device vectors are torch tensors on a HIP device (PyTorch provides device
memory and streams); host inputs are numpy arrays.  The binding fails loudly
when the library has not been built -- there is no CPU fallback.

The function names are those of the C ABI (include/tbh.h) without the
``tbh_`` prefix.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtbh.so")

TBH_OK, TBH_EINVAL, TBH_ENOMEM, TBH_EHIP, TBH_ENOCONV, TBH_ESTATE = 0, -1, -2, -3, -4, -5
TBH_SP3S, TBH_SP3D5S = 0, 1
TBH_F64, TBH_F32 = 0, 1


class TBHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tbh error {code}: {msg}")
        self.code = code


class tbh_geometry(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("pos_q", C.POINTER(C.c_int32)),
                ("species", C.POINTER(C.c_uint8)), ("box_q", C.c_int32 * 3),
                ("periodic", C.c_int32 * 3)]


class tbh_params(C.Structure):
    _fields_ = [("model", C.c_int32), ("spin", C.c_int32), ("n_species", C.c_int32),
                ("onsite", C.POINTER(C.c_double)), ("sk", C.POINTER(C.c_double)),
                ("so_delta", C.POINTER(C.c_double)), ("passivation_eV", C.c_double)]


class tbh_build_opts(C.Structure):
    _fields_ = [("bond_scale", C.POINTER(C.c_double)), ("onsite_pot", C.POINTER(C.c_double)),
                ("kfrac", C.POINTER(C.c_double)), ("prec", C.c_int32),
                ("lanes_per_atom", C.c_int32), ("keep_f64", C.c_int32),
                ("multi_vector", C.c_int32), ("tabulated", C.c_int32), ("spin_diagonal", C.c_int32)]


class tbh_ham_info(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("dim", C.c_int64), ("n_orb", C.c_int32),
                ("is_complex", C.c_int32), ("prec", C.c_int32), ("lanes_per_atom", C.c_int32),
                ("onsite_diagonal", C.c_int32), ("has_f64", C.c_int32),
                ("n_dangling", C.c_int64), ("stored_bytes", C.c_int64), ("hx_bytes", C.c_int64),
                ("tabulated", C.c_int32), ("spin_diagonal", C.c_int32)]


class tbh_lanczos_opts(C.Structure):
    _fields_ = [("sigma", C.c_double), ("k", C.c_int32), ("max_iter", C.c_int32),
                ("reorth", C.c_int32), ("n_cand", C.c_int32), ("res_tol", C.c_double),
                ("merge_tol", C.c_double), ("v0", C.POINTER(C.c_double)),
                ("v0_dev", C.c_void_p)]


class tbh_lanczos_report(C.Structure):
    _fields_ = [("steps", C.c_int32), ("breakdown", C.c_int32), ("n_found", C.c_int32),
                ("n_cand", C.c_int32), ("max_res", C.c_double), ("seconds", C.c_double),
                ("hx_seconds", C.c_double)]


class tbh_block_lanczos_opts(C.Structure):
    _fields_ = [("sigma", C.c_double), ("block", C.c_int32), ("steps", C.c_int32), ("cycles", C.c_int32),
                ("k", C.c_int32), ("res_tol", C.c_double), ("defl_tol", C.c_double), ("x0_dev", C.c_void_p),
                ("fold", C.c_int32)]


class tbh_block_lanczos_report(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("n_found", C.c_int32), ("deflated", C.c_int32),
                ("max_res", C.c_double), ("seconds", C.c_double), ("hx_seconds", C.c_double)]


class tbh_filter_opts(C.Structure):
    _fields_ = [("sigma", C.c_double), ("block", C.c_int32), ("degree", C.c_int32), ("degree_cold", C.c_int32),
                ("max_iter", C.c_int32), ("k", C.c_int32), ("res_tol", C.c_double), ("x0_dev", C.c_void_p)]


class tbh_filter_report(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("n_found", C.c_int32), ("max_res", C.c_double), ("emin", C.c_double),
                ("emax", C.c_double), ("seconds", C.c_double)]


class tbh_scf_opts(C.Structure):
    _fields_ = [("grid", C.c_int32 * 3), ("h_nm", C.c_double), ("eps_r", C.c_double),
                ("T_K", C.c_double), ("mix_alpha", C.c_double), ("tol_eV", C.c_double),
                ("sigma_mid", C.c_double), ("e_cbm", C.c_double), ("fermi_fixed", C.c_double),
                ("n_cand", C.c_int32), ("lanczos_iter", C.c_int32), ("res_tol", C.c_double),
                ("cg_tol", C.c_double), ("cg_max_iter", C.c_int32),
                ("donor_atoms", C.POINTER(C.c_int32)), ("n_donors", C.c_int32),
                ("v0", C.POINTER(C.c_double)), ("eig_mode", C.c_int32), ("block", C.c_int32),
                ("filter_degree", C.c_int32), ("filter_degree_cold", C.c_int32), ("filter_max_iter", C.c_int32),
                ("k_states", C.c_int32), ("e_vbm", C.c_double), ("update_mode", C.c_int32),
                ("newton_states", C.c_int32), ("newton_kT", C.c_double), ("anderson_depth", C.c_int32),
                ("newton_cg_tol", C.c_double), ("newton_cg_max_iter", C.c_int32),
                ("filter_max_iter_cold", C.c_int32)]


class tbh_scf_report(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double),
                ("fermi", C.c_double), ("n_cb", C.c_int32), ("n_conv", C.c_int32),
                ("electrons", C.c_double), ("cg_iters", C.c_int32), ("cg_rel_res", C.c_double),
                ("lanczos_steps", C.c_int32), ("u_min", C.c_double), ("sigma", C.c_double),
                ("seconds", C.c_double),
                ("eig_seconds", C.c_double), ("poisson_seconds", C.c_double), ("fell_back", C.c_int32),
                ("newton_cg_iters", C.c_int32), ("newton_pairs", C.c_int32), ("newton_seconds", C.c_double)]


class tbh_scf_start(C.Structure):
    _fields_ = [("kind", C.c_int32), ("net", C.c_void_p), ("mean_dev", C.c_void_p), ("scale", C.c_double),
                ("feat_scale", C.c_double), ("symmetrize", C.c_int32), ("first_res_limit", C.c_double)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_SIGS = [
    ("tbh_version", C.c_int, []),
    ("tbh_last_error", C.c_char_p, []),
    ("tbh_ctx_create", C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("tbh_ctx_destroy", C.c_int, [C.c_void_p]),
    ("tbh_ctx_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_build_blocks_host", C.c_int, [C.POINTER(tbh_geometry), C.POINTER(tbh_params),
                                        C.POINTER(tbh_build_opts), C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    ("tbh_tabulate_host", C.c_int, [C.POINTER(tbh_geometry), C.POINTER(tbh_params),
                                    C.POINTER(tbh_build_opts), C.c_void_p, C.c_int64,
                                    C.POINTER(C.c_int32), C.c_void_p]),
    ("tbh_build_hamiltonian", C.c_int, [C.c_void_p, C.POINTER(tbh_geometry), C.POINTER(tbh_params),
                                        C.POINTER(tbh_build_opts), C.POINTER(C.c_void_p)]),
    ("tbh_ham_destroy", C.c_int, [C.c_void_p]),
    ("tbh_ham_info_get", C.c_int, [C.c_void_p, C.POINTER(tbh_ham_info)]),
    ("tbh_ham_neighbours", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("tbh_ham_set_potential", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_apply_h", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("tbh_apply_h_f64", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("tbh_lanczos_eigs", C.c_int, [C.c_void_p, C.POINTER(tbh_lanczos_opts), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(tbh_lanczos_report)]),
    ("tbh_lanczos_run", C.c_int, [C.c_void_p, C.POINTER(tbh_lanczos_opts), C.c_void_p,
                                  C.c_void_p, C.c_int32, C.POINTER(tbh_lanczos_report)]),
    ("tbh_tridiag_eig", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("tbh_block_lanczos_eigs", C.c_int, [C.c_void_p, C.POINTER(tbh_block_lanczos_opts), C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.POINTER(tbh_block_lanczos_report)]),
    ("tbh_filtered_eigs", C.c_int, [C.c_void_p, C.POINTER(tbh_filter_opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(tbh_filter_report)]),
    ("tbh_symm_eig_near", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_int32, C.c_void_p,
                                    C.c_void_p]),
    ("tbh_poisson_solve", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("tbh_poisson_solve_noalloc", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_double, C.c_double,
                                            C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                            C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("tbh_scf_create", C.c_int, [C.c_void_p, C.POINTER(tbh_scf_opts), C.POINTER(C.c_void_p)]),
    ("tbh_scf_destroy", C.c_int, [C.c_void_p]),
    ("tbh_scf_set_potential", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_scf_get_potential", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_scf_step", C.c_int, [C.c_void_p, C.POINTER(tbh_scf_report)]),
    ("tbh_scf_get_density", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_scf_set_start", C.c_int, [C.c_void_p, C.POINTER(tbh_scf_start)]),
    ("tbh_scf_run", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(tbh_scf_report)]),
    ("tbh_apply_h_multi", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    ("tbh_batch_create", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    ("tbh_batch_destroy", C.c_int, [C.c_void_p]),
    ("tbh_batch_apply", C.c_int, [C.c_void_p]),
    ("tbh_batch_apply_separate", C.c_int, [C.c_void_p]),
    ("tbh_batch_autotune", C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]),
    ("tbh_batch_configure", C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    ("tbh_net_create", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), C.POINTER(C.c_void_p)]),
    ("tbh_net_set_loss_weights", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_net_destroy", C.c_int, [C.c_void_p]),
    ("tbh_net_num_params", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("tbh_net_set_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_net_get_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("tbh_net_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("tbh_net_gradients", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    ("tbh_net_train_step", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32,
                                     C.c_double, C.POINTER(C.c_double)]),
]


def lib():
    """Load libtbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1003_4570_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def _check(rc):
    if rc != TBH_OK:
        raise TBHError(rc, lib().tbh_last_error().decode())


def _dptr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def last_error() -> str:
    return lib().tbh_last_error().decode()


def version() -> int:
    return lib().tbh_version()


class _Inputs:
    """Host arrays kept alive for the duration of one call."""

    def __init__(self, pos_q, species, box_q, periodic, model, spin, onsite, sk,
                 so_delta=None, passivation_eV=0.0, bond_scale=None, onsite_pot=None,
                 kfrac=None, prec=TBH_F32, lanes_per_atom=0, keep_f64=False, n_species=None,
                 multi_vector=False, tabulated=False, spin_diagonal=False):
        self.pos = _dptr(pos_q, np.int32).reshape(-1, 3)
        self.spc = _dptr(species, np.uint8).ravel()
        self.onsite = _dptr(onsite, np.float64)
        self.sk = _dptr(sk, np.float64)
        ns = int(self.onsite.shape[0]) if n_species is None else int(n_species)
        self.so = None if so_delta is None else _dptr(so_delta, np.float64)
        self.bs = None if bond_scale is None else _dptr(bond_scale, np.float64)
        self.pot = None if onsite_pot is None else _dptr(onsite_pot, np.float64)
        self.kf = None if kfrac is None else _dptr(kfrac, np.float64)
        if isinstance(prec, str):
            prec = TBH_F64 if prec == "f64" else TBH_F32
        self.g = tbh_geometry(self.pos.shape[0], _p(self.pos, C.c_int32), _p(self.spc, C.c_uint8),
                              (C.c_int32 * 3)(*[int(b) for b in box_q]),
                              (C.c_int32 * 3)(*[int(b) for b in periodic]))
        self.par = tbh_params(int(model), int(spin), ns, _p(self.onsite, C.c_double),
                              _p(self.sk, C.c_double), _p(self.so, C.c_double), float(passivation_eV))
        self.opt = tbh_build_opts(_p(self.bs, C.c_double), _p(self.pot, C.c_double),
                                  _p(self.kf, C.c_double), int(prec), int(lanes_per_atom),
                                  int(bool(keep_f64)), int(bool(multi_vector)), int(bool(tabulated)),
                                  int(bool(spin_diagonal)))
        self.n = self.pos.shape[0]
        self.n_o = (5 if int(model) == TBH_SP3S else 10) * (2 if spin else 1)


def problem_args(prob, prec=None, **kw):
    """Keyword arguments of build_hamiltonian for a workloads.Problem-like
    object (attributes pos_q, species, box_q, periodic, params, bond_scale,
    onsite_pot, kfrac, prec)."""
    par = prob.params
    d = dict(pos_q=prob.pos_q, species=prob.species, box_q=prob.box_q, periodic=prob.periodic,
             model=par["model"], spin=par["spin"], onsite=par["onsite"], sk=par["sk"],
             so_delta=par["so_delta"], passivation_eV=par["passivation_eV"],
             bond_scale=prob.bond_scale, onsite_pot=prob.onsite_pot, kfrac=prob.kfrac,
             prec=prob.prec if prec is None else prec)
    d.update(kw)
    return d


def build_blocks_host(**kw):
    """Host-only build step: (nbr [n,4], wrap [n,4,3], onsite, bonds, complex).
    onsite [n, n_o, n_o] and bonds [n, 4, n_o, n_o] are float64 or complex128."""
    a = _Inputs(**kw)
    n, no = a.n, a.n_o
    nbr = np.empty((n, 4), np.int32)
    wrap = np.empty((n, 4, 3), np.int8)
    isc = C.c_int32(0)
    _check(lib().tbh_build_blocks_host(C.byref(a.g), C.byref(a.par), C.byref(a.opt),
                                       nbr.ctypes.data, wrap.ctypes.data, None, None, C.byref(isc)))
    cs = 2 if isc.value else 1
    on = np.empty(n * no * no * cs)
    bd = np.empty(n * 4 * no * no * cs)
    _check(lib().tbh_build_blocks_host(C.byref(a.g), C.byref(a.par), C.byref(a.opt),
                                       None, None, on.ctypes.data, bd.ctypes.data, None))
    if cs == 2:
        on = on.view(np.complex128)
        bd = bd.view(np.complex128)
    return nbr, wrap, on.reshape(n, no, no), bd.reshape(n, 4, no, no), bool(isc.value)


def tabulate_host(**kw):
    """Host-only tabulated build step: (blocks [nu, n_o, n_o], on-site
    diagonals [n_species, n_o], key records [n, 8] uint8) in caller order."""
    a = _Inputs(**kw)
    nu = C.c_int32(0)
    _check(lib().tbh_tabulate_host(C.byref(a.g), C.byref(a.par), C.byref(a.opt), None, 0,
                                   C.byref(nu), None))
    no, ns = a.n_o, int(a.par.n_species)
    table = np.empty(nu.value * no * no + ns * no)
    keys = np.empty((a.n, 8), np.uint8)
    _check(lib().tbh_tabulate_host(C.byref(a.g), C.byref(a.par), C.byref(a.opt), table.ctypes.data,
                                   table.size, C.byref(nu), keys.ctypes.data))
    k = nu.value * no * no
    return table[:k].reshape(nu.value, no, no), table[k:].reshape(ns, no), keys


class _Handle:
    """A library object.  close() first closes the objects that depend on it
    (an SCF loop before its Hamiltonian, everything before its Context), so
    the library never reaches a destroyed parent, whatever order Python
    finalises the objects in (reference cycles at interpreter exit)."""

    _destroy = ""

    def _adopt(self, *parents):
        self._deps = weakref.WeakSet()
        for p in parents:
            p._deps.add(self)

    def close(self):
        for d in list(getattr(self, "_deps", ())):
            d.close()
        if getattr(self, "h", None):
            getattr(lib(), self._destroy)(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context(_Handle):
    """A library context on one HIP device and stream."""

    _destroy = "tbh_ctx_destroy"

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._adopt()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = C.c_void_p()
        _check(lib().tbh_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h


class Hamiltonian(_Handle):
    """A device Hamiltonian built by tbh_build_hamiltonian."""

    _destroy = "tbh_ham_destroy"

    def __init__(self, ctx: Context, handle):
        self._adopt(ctx)
        self.ctx = ctx
        self.h = handle
        info = tbh_ham_info()
        _check(lib().tbh_ham_info_get(self.h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in tbh_ham_info._fields_}

    @property
    def dim(self):
        return self.info["dim"]

    @property
    def is_complex(self):
        return bool(self.info["is_complex"])

    @property
    def prec(self):
        return self.info["prec"]

    def torch_dtype(self, f64=False):
        import torch
        if self.prec == TBH_F64 or f64:
            return torch.complex128 if self.is_complex else torch.float64
        return torch.complex64 if self.is_complex else torch.float32


def build_hamiltonian(ctx: Context, **kw) -> Hamiltonian:
    """Build H on the context's device (see problem_args for the keywords)."""
    a = _Inputs(**kw)
    h = C.c_void_p()
    _check(lib().tbh_build_hamiltonian(ctx.h, C.byref(a.g), C.byref(a.par), C.byref(a.opt), C.byref(h)))
    return Hamiltonian(ctx, h)


def ham_neighbours(ham: Hamiltonian):
    n = ham.info["n_atoms"]
    nbr = np.empty((n, 4), np.int32)
    wrap = np.empty((n, 4, 3), np.int8)
    _check(lib().tbh_ham_neighbours(ham.h, nbr.ctypes.data, wrap.ctypes.data))
    return nbr, wrap


def _check_vec(ham, t, f64=False):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device vectors must be torch tensors on a HIP device")
    if t.dtype != ham.torch_dtype(f64):
        raise TypeError(f"expected dtype {ham.torch_dtype(f64)}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("vectors must be contiguous")


def ham_set_potential(ham: Hamiltonian, pot):
    """pot: float64 device tensor [n_atoms] (eV) or None."""
    if pot is None:
        _check(lib().tbh_ham_set_potential(ham.h, None))
        return
    import torch
    assert pot.dtype == torch.float64 and pot.is_cuda and pot.numel() == ham.info["n_atoms"]
    _check(lib().tbh_ham_set_potential(ham.h, C.c_void_p(pot.data_ptr())))


def apply_h(ham: Hamiltonian, x, y=None):
    """y = H x on the device (x, y: [dim] tensors of the ham's dtype)."""
    import torch
    _check_vec(ham, x)
    if y is None:
        y = torch.empty_like(x)
    _check_vec(ham, y)
    if x.numel() != ham.dim or y.numel() != ham.dim:
        raise ValueError("vector length must equal dim")
    _check(lib().tbh_apply_h(ham.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), 1))
    return y


def apply_h_f64(ham: Hamiltonian, x, y=None):
    """y = H x in FP64 with the FP64 copy of H."""
    import torch
    _check_vec(ham, x, f64=True)
    if y is None:
        y = torch.empty_like(x)
    _check_vec(ham, y, f64=True)
    _check(lib().tbh_apply_h_f64(ham.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
    return y


def _report(r):
    return {k: getattr(r, k) for k, _ in tbh_lanczos_report._fields_}


def _v0_args(ham, v0):
    """(host array or None, device pointer or None) for a start vector given
    as a numpy array (host) or an FP64 / complex128 device tensor."""
    try:
        import torch
        if isinstance(v0, torch.Tensor):
            if not v0.is_cuda or v0.dtype not in (torch.float64, torch.complex128) or not v0.is_contiguous():
                raise TypeError("device start vector must be a contiguous float64/complex128 tensor")
            if v0.numel() * (2 if v0.is_complex() else 1) != ham.dim * (2 if ham.is_complex else 1):
                raise ValueError("start vector length must equal dim")
            return None, C.c_void_p(v0.data_ptr())
    except ImportError:
        pass
    return _v0_host(ham, v0), None


def _v0_host(ham, v0):
    v = np.asarray(v0)
    if np.iscomplexobj(v):
        v = np.ascontiguousarray(v, dtype=np.complex128).view(np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    if v.size != ham.dim * (2 if ham.is_complex else 1):
        raise ValueError("start vector length must equal dim (complex: 2*dim reals)")
    return v


def lanczos_run(ham: Hamiltonian, m: int, v0, reorth: bool = False, time_hx: bool = False):
    """The Lanczos recurrence alone (m steps).  Returns (alpha, beta, report)
    with beta[j] = beta_{j+1}."""
    v, vd = _v0_args(ham, v0)
    o = tbh_lanczos_opts(0.0, 1, int(m), int(bool(reorth)), 0, 0.0, 0.0,
                         None if v is None else v.ctypes.data_as(C.POINTER(C.c_double)), vd)
    a = np.zeros(m)
    b = np.zeros(m)
    rep = tbh_lanczos_report()
    _check(lib().tbh_lanczos_run(ham.h, C.byref(o), a.ctypes.data, b.ctypes.data,
                                 int(bool(time_hx)), C.byref(rep)))
    r = _report(rep)
    return a[:r["steps"]], b[:r["steps"]], r


def lanczos_eigs(ham: Hamiltonian, sigma: float, k: int, max_iter: int, v0, reorth: bool = True,
                 n_cand: int = 0, res_tol: float = 0.0, merge_tol: float = 0.0,
                 want_vectors: bool = False, allow_partial: bool = True):
    """Distinct converged eigenvalues nearest sigma.  Returns a dict with
    evals (raw Ritz values), refined (FP64 Rayleigh quotients), res, copies,
    report, and vectors ([k, dim] FP64/complex128 device tensor) if asked."""
    import torch
    v, vd = _v0_args(ham, v0)
    o = tbh_lanczos_opts(float(sigma), int(k), int(max_iter), int(bool(reorth)), int(n_cand),
                         float(res_tol), float(merge_tol),
                         None if v is None else v.ctypes.data_as(C.POINTER(C.c_double)), vd)
    ev = np.zeros(k)
    rf = np.zeros(k)
    rs = np.zeros(k)
    cp = np.zeros(k, np.int32)
    vec = None
    if want_vectors:
        vec = torch.zeros((k, ham.dim), dtype=torch.complex128 if ham.is_complex else torch.float64,
                          device=f"cuda:{ham.ctx.device}")
    rep = tbh_lanczos_report()
    rc = lib().tbh_lanczos_eigs(ham.h, C.byref(o), ev.ctypes.data, rf.ctypes.data, rs.ctypes.data,
                                cp.ctypes.data, None if vec is None else C.c_void_p(vec.data_ptr()),
                                C.byref(rep))
    if rc != TBH_OK and not (allow_partial and rc == TBH_ENOCONV):
        _check(rc)
    r = _report(rep)
    n = r["n_found"]
    out = dict(evals=ev[:n], refined=rf[:n], res=rs[:n], copies=cp[:n], report=r, status=rc)
    if vec is not None:
        out["vectors"] = vec[:n]
    return out


def block_lanczos_eigs(ham: Hamiltonian, sigma: float, k: int, block: int, steps: int, cycles: int = 1,
                       x0=None, res_tol: float = 0.0, defl_tol: float = 0.0, want_vectors: bool = False,
                       allow_partial: bool = True, fold: bool = False):
    """The k converged Ritz pairs nearest sigma by block Lanczos (each copy of
    a repeated eigenvalue counts).  x0: None (SplitMix64 block) or a [block,
    dim] float64 device tensor.  fold: Krylov space of (H - sigma)^2.
    Returns dict(evals, refined, res, report[, vectors [n_found, dim] float64
    device tensor])."""
    import torch
    if x0 is not None:
        if not (isinstance(x0, torch.Tensor) and x0.is_cuda and x0.dtype == torch.float64 and x0.is_contiguous()
                and x0.numel() == block * ham.dim):
            raise TypeError("x0 must be a contiguous float64 device tensor [block, dim]")
    o = tbh_block_lanczos_opts(float(sigma), int(block), int(steps), int(cycles), int(k), float(res_tol),
                               float(defl_tol), None if x0 is None else C.c_void_p(x0.data_ptr()),
                               int(bool(fold)))
    ev = np.zeros(k)
    rf = np.zeros(k)
    rs = np.zeros(k)
    vec = None
    if want_vectors:
        vec = torch.zeros((k, ham.dim), dtype=torch.float64, device=f"cuda:{ham.ctx.device}")
    rep = tbh_block_lanczos_report()
    rc = lib().tbh_block_lanczos_eigs(ham.h, C.byref(o), ev.ctypes.data, rf.ctypes.data, rs.ctypes.data,
                                      None if vec is None else C.c_void_p(vec.data_ptr()), C.byref(rep))
    if rc != TBH_OK and not (allow_partial and rc == TBH_ENOCONV):
        _check(rc)
    r = {f: getattr(rep, f) for f, _ in rep._fields_}
    n = r["n_found"]
    out = dict(evals=ev[:n], refined=rf[:n], res=rs[:n], report=r, status=rc)
    if vec is not None:
        out["vectors"] = vec[:n]
    return out


def filtered_eigs(ham: Hamiltonian, sigma: float, k: int, block: int = 64, degree: int = 20, degree_cold: int = 60,
                  max_iter: int = 50, res_tol: float = 0.0, x0=None, want_vectors: bool = False,
                  allow_partial: bool = True):
    """The k converged pairs nearest sigma (sigma in a gap) by Chebyshev-filtered
    subspace iteration on (H - sigma)^2.  x0: None or a [block, dim] float64
    device tensor.  Returns dict(evals, res, report[, vectors])."""
    import torch
    if x0 is not None and not (isinstance(x0, torch.Tensor) and x0.is_cuda and x0.dtype == torch.float64
                               and x0.is_contiguous() and x0.numel() == block * ham.dim):
        raise TypeError("x0 must be a contiguous float64 device tensor [block, dim]")
    o = tbh_filter_opts(float(sigma), int(block), int(degree), int(degree_cold), int(max_iter), int(k),
                        float(res_tol), None if x0 is None else C.c_void_p(x0.data_ptr()))
    ev = np.zeros(k)
    rs = np.zeros(k)
    vec = None
    if want_vectors:
        vec = torch.zeros((k, ham.dim), dtype=torch.float64, device=f"cuda:{ham.ctx.device}")
    rep = tbh_filter_report()
    rc = lib().tbh_filtered_eigs(ham.h, C.byref(o), ev.ctypes.data, rs.ctypes.data,
                                 None if vec is None else C.c_void_p(vec.data_ptr()), C.byref(rep))
    if rc != TBH_OK and not (allow_partial and rc == TBH_ENOCONV):
        _check(rc)
    r = {f: getattr(rep, f) for f, _ in rep._fields_}
    n = r["n_found"]
    out = dict(evals=ev[:n], res=rs[:n], report=r, status=rc)
    if vec is not None:
        out["vectors"] = vec[:n]
    return out


def symm_eig_near(ctx: Context, A, sigma: float, nc: int):
    """The nc eigenpairs nearest sigma of the real symmetric matrix A (host
    array) with the device's projected-matrix eigensolver.  Returns (theta
    ascending, vectors [nc, n])."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    th = np.zeros(nc)
    V = np.zeros((nc, n))
    _check(lib().tbh_symm_eig_near(ctx.h, n, A.ctypes.data, float(sigma), int(nc), th.ctypes.data, V.ctypes.data))
    return th, V


def tridiag_eig(ctx: Context, diag, off):
    """Eigenvalues (ascending) of a symmetric tridiagonal matrix, FP64
    bisection on the device."""
    d = np.ascontiguousarray(diag, dtype=np.float64)
    e = np.ascontiguousarray(off, dtype=np.float64)
    th = np.zeros(d.size)
    _check(lib().tbh_tridiag_eig(ctx.h, d.size, d.ctypes.data, e.ctypes.data if e.size else None,
                                 th.ctypes.data))
    return th


def poisson_solve(ctx: Context, grid, h_nm, eps_r, rho, phi=None, rel_tol=1e-10, max_iter=100000,
                  noalloc=False):
    """FP64 CG for -eps0 eps_r Lap_h phi = rho on the device.  rho: [nz, ny, nx]
    float64 device tensor (e/nm^3); phi: initial guess (updated in place) or
    None (zero).  noalloc selects the entry point that allocates no device
    memory (grids up to 2^18 nodes).  Returns (phi, iterations, relative
    residual)."""
    import torch
    if phi is None:
        phi = torch.zeros_like(rho)
    for t in (rho, phi):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == int(np.prod(grid))):
            raise TypeError("rho and phi must be contiguous float64 device tensors of the grid's size")
    g = (C.c_int32 * 3)(*[int(v) for v in grid])
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    fn = lib().tbh_poisson_solve_noalloc if noalloc else lib().tbh_poisson_solve
    rc = fn(ctx.h, g, float(h_nm), float(eps_r), C.c_void_p(rho.data_ptr()),
            C.c_void_p(phi.data_ptr()), float(rel_tol), int(max_iter),
            C.byref(it), C.byref(rr))
    if rc not in (TBH_OK, TBH_ENOCONV):
        _check(rc)
    return phi, it.value, rr.value


class SCF(_Handle):
    """Self-consistent Schrodinger-Poisson loop on a device Hamiltonian."""

    _destroy = "tbh_scf_destroy"

    def __init__(self, ham: Hamiltonian, grid, donor_atoms, v0, sigma_mid, e_cbm, h_nm, eps_r=11.7,
                 T_K=4.0, mix_alpha=0.1, tol_eV=1e-4, n_cand=48, lanczos_iter=600, res_tol=1e-4,
                 cg_tol=1e-12, cg_max_iter=20000, fermi_fixed=None, eig_mode=0, block=64, filter_degree=20,
                 filter_degree_cold=60, filter_max_iter=20, k_states=40, e_vbm=float("nan"), update_mode=0,
                 newton_states=64, newton_kT=0.01, anderson_depth=4, newton_cg_tol=1e-6,
                 newton_cg_max_iter=20000, filter_max_iter_cold=0):
        self._adopt(ham)
        self.ham = ham
        self.grid = tuple(int(g) for g in grid)
        self._donors = np.ascontiguousarray(donor_atoms, dtype=np.int32)
        self._v0 = _v0_host(ham, v0)
        o = tbh_scf_opts((C.c_int32 * 3)(*self.grid), float(h_nm), float(eps_r), float(T_K),
                         float(mix_alpha), float(tol_eV), float(sigma_mid), float(e_cbm),
                         float("nan") if fermi_fixed is None else float(fermi_fixed),
                         int(n_cand), int(lanczos_iter), float(res_tol), float(cg_tol),
                         int(cg_max_iter), _p(self._donors, C.c_int32), int(self._donors.size),
                         self._v0.ctypes.data_as(C.POINTER(C.c_double)), int(eig_mode), int(block),
                         int(filter_degree), int(filter_degree_cold), int(filter_max_iter), int(k_states),
                         float(e_vbm), int(update_mode), int(newton_states), float(newton_kT),
                         int(anderson_depth), float(newton_cg_tol), int(newton_cg_max_iter),
                         int(filter_max_iter_cold))
        h = C.c_void_p()
        _check(lib().tbh_scf_create(ham.h, C.byref(o), C.byref(h)))
        self.h = h

    def set_potential(self, U=None):
        """U: [nz, ny, nx] float64 device tensor (eV) or None (zero start)."""
        _check(lib().tbh_scf_set_potential(self.h, None if U is None else C.c_void_p(U.data_ptr())))

    def potential(self):
        import torch
        nx, ny, nz = self.grid
        U = torch.empty((nz, ny, nx), dtype=torch.float64, device=f"cuda:{self.ham.ctx.device}")
        _check(lib().tbh_scf_get_potential(self.h, C.c_void_p(U.data_ptr())))
        return U

    def set_start(self, kind, net=None, mean=None, scale=0.0, feat_scale=1.0, symmetrize=True,
                  first_res_limit=0.0):
        """Start potential built on the device (tbh_scf_set_start): kind
        "zero", "mean" (U_bare + mean) or "learned" (U_bare + mean + scale *
        the network's output, averaged over the point operations).  mean:
        float32 device tensor [nz, ny, nx]."""
        k = {"zero": 0, "mean": 1, "learned": 2}[kind]
        if mean is not None:
            self._mean = mean.float().contiguous()
        o = tbh_scf_start(k, None if net is None else net.h, None if mean is None else C.c_void_p(self._mean.data_ptr()),
                          float(scale), float(feat_scale), int(bool(symmetrize)), float(first_res_limit))
        _check(lib().tbh_scf_set_start(self.h, C.byref(o)))

    def density(self):
        """Electrons per atom of the last step (float64 device tensor, caller order)."""
        import torch
        n = torch.empty(self.ham.info["n_atoms"], dtype=torch.float64, device=f"cuda:{self.ham.ctx.device}")
        _check(lib().tbh_scf_get_density(self.h, C.c_void_p(n.data_ptr())))
        return n

    def step(self):
        r = tbh_scf_report()
        _check(lib().tbh_scf_step(self.h, C.byref(r)))
        return {k: getattr(r, k) for k, _ in tbh_scf_report._fields_}

    def run(self, max_iter):
        r = tbh_scf_report()
        rc = lib().tbh_scf_run(self.h, int(max_iter), C.byref(r))
        if rc not in (TBH_OK, TBH_ENOCONV):
            _check(rc)
        return {k: getattr(r, k) for k, _ in tbh_scf_report._fields_}



def _check_mv(ham, t, nrhs):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError("multi-vectors must be contiguous device tensors")
    want = torch.complex64 if ham.is_complex else torch.float32
    if t.dtype != want or t.numel() != ham.dim * nrhs:
        raise TypeError(f"expected {want} [dim, nrhs] = [{ham.dim}, {nrhs}]")


def apply_h_multi(ham: Hamiltonian, X, Y=None):
    """Y = H X on the matrix cores.  X: [dim, nrhs] complex64 / float32
    device tensor (nrhs = 16 or 32)."""
    import torch
    nrhs = X.shape[-1]
    _check_mv(ham, X, nrhs)
    if Y is None:
        Y = torch.empty_like(X)
    _check_mv(ham, Y, nrhs)
    _check(lib().tbh_apply_h_multi(ham.h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), int(nrhs)))
    return Y


class Batch(_Handle):
    """Many Hamiltonians' multi-vector products in one persistent launch
    (captured in a HIP graph)."""

    _destroy = "tbh_batch_destroy"

    def __init__(self, ctx: Context, hams, Xs, Ys):
        nrhs = Xs[0].shape[-1]
        for h, x, y in zip(hams, Xs, Ys):
            _check_mv(h, x, nrhs)
            _check_mv(h, y, nrhs)
        self._adopt(ctx, *hams)
        self.ctx, self.hams, self.Xs, self.Ys = ctx, list(hams), list(Xs), list(Ys)
        n = len(hams)
        H = (C.c_void_p * n)(*[h.h for h in hams])
        X = (C.c_void_p * n)(*[x.data_ptr() for x in Xs])
        Y = (C.c_void_p * n)(*[y.data_ptr() for y in Ys])
        b = C.c_void_p()
        _check(lib().tbh_batch_create(ctx.h, H, n, X, Y, int(nrhs), C.byref(b)))
        self.h = b

    def apply(self):
        _check(lib().tbh_batch_apply(self.h))

    def apply_separate(self):
        _check(lib().tbh_batch_apply_separate(self.h))

    def configure(self, grid, remap):
        _check(lib().tbh_batch_configure(self.h, int(grid), int(remap)))

    def autotune(self, cache_path=None):
        g = C.c_int32(0)
        r = C.c_int32(0)
        ms = C.c_double(0)
        _check(lib().tbh_batch_autotune(self.h, None if cache_path is None else str(cache_path).encode(),
                                        C.byref(g), C.byref(r), C.byref(ms)))
        return dict(grid=g.value, remap=r.value, ms=ms.value)



class Net(_Handle):
    """The convolutional start-potential surrogate (device kernels).
    grid = (nx, ny, nz); inputs are float32 device tensors [in_channels, nz,
    ny, nx] (or [nz, ny, nx] for one channel), outputs [nz, ny, nx]."""

    _destroy = "tbh_net_destroy"

    def __init__(self, ctx: Context, grid, channels=32, in_channels=1, dilations=(1, 2, 4, 1)):
        self._adopt(ctx)
        self.ctx = ctx
        self.grid = tuple(int(g) for g in grid)
        self.in_channels = int(in_channels)
        self.dilations = tuple(int(d) for d in dilations)
        nl = len(self.dilations)
        h = C.c_void_p()
        _check(lib().tbh_net_create(ctx.h, int(channels), self.in_channels, nl, (C.c_int32 * nl)(*self.dilations),
                                    (C.c_int32 * 3)(*self.grid), C.byref(h)))
        self.h = h
        n = C.c_int64(0)
        _check(lib().tbh_net_num_params(self.h, C.byref(n)))
        self.n_params = n.value

    def set_params(self, flat):
        w = np.ascontiguousarray(flat, dtype=np.float32).ravel()
        assert w.size == self.n_params
        _check(lib().tbh_net_set_params(self.h, w.ctypes.data))

    def get_params(self):
        w = np.empty(self.n_params, np.float32)
        _check(lib().tbh_net_get_params(self.h, w.ctypes.data))
        return w

    def _chk(self, t, channels=1):
        import torch
        nx, ny, nz = self.grid
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                and t.is_contiguous() and t.numel() == channels * nx * ny * nz):
            raise TypeError(f"maps must be contiguous float32 device tensors [{channels}, nz, ny, nx]")

    def set_loss_weights(self, w):
        """Per-voxel training-loss weights (float32 device [nz, ny, nx]) or None."""
        if w is not None:
            self._chk(w)
        _check(lib().tbh_net_set_loss_weights(self.h, None if w is None else C.c_void_p(w.data_ptr())))

    def forward(self, x, y=None):
        import torch
        self._chk(x, self.in_channels)
        if y is None:
            nx, ny, nz = self.grid
            y = torch.empty((nz, ny, nx), dtype=torch.float32, device=x.device)
        self._chk(y)
        _check(lib().tbh_net_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def gradients(self, x, t):
        self._chk(x, self.in_channels)
        self._chk(t)
        g = np.empty(self.n_params, np.float32)
        loss = C.c_double(0)
        _check(lib().tbh_net_gradients(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                       g.ctypes.data, C.byref(loss)))
        return g, loss.value

    def train_step(self, xs, ts, lr=1e-3):
        for a in xs:
            self._chk(a, self.in_channels)
        for a in ts:
            self._chk(a)
        n = len(xs)
        X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        T = (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        loss = C.c_double(0)
        _check(lib().tbh_net_train_step(self.h, X, T, n, float(lr), C.byref(loss)))
        return loss.value



def flatten_params(params):
    """Canonical flat parameter vector from [(W [co, ci, 3, 3, 3], b [co])]."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflatten_params(flat, channels=32, in_channels=1, n_layers=4):
    shapes = [(channels, in_channels)] + [(channels, channels)] * (n_layers - 2) + [(1, channels)]
    out, o = [], 0
    for co, ci in shapes:
        nW = co * ci * 27
        W = np.asarray(flat[o:o + nW], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        o += nW
        b = np.asarray(flat[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out
