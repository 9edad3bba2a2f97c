"""Python binding of libhub (include/hub.h): argument marshalling only.

Every step of the time evolution runs in the HIP library; this module turns
Python objects into the C structs and raw device pointers the ABI expects.
Device vectors are torch tensors (complex128 for HUB_C128, complex64 for
HUB_C64) on the handle's GPU; torch supplies the memory and the stream.

The library is loaded from this package directory (libhub.so, built by
`paper_2005_13498_amd.build`).  If it is missing, every call raises.

Typical use (12-site cluster, ground state, midpoint steps under a pulse):

    import torch, paper_2005_13498_amd as hub
    from synth import cluster_2d, PulseParams
    B = hub.Basis(cluster_2d(3, 4), 8.0, 6, 6, device=0)
    pulse = PulseParams(0, 0.9, 8.0, 2.5, 0.5)          # kind, A0, omega, t0, sigma
    v = torch.empty(B.dim, dtype=torch.complex128, device="cuda:0")
    hub.hub_ground_state(B.handle, hub.hub_pulse_A(pulse, 0.0), v, hub.make_opts(tol=1e-12, m_max=100))
    st, obs, log = hub.hub_propagate(B.handle, [pulse], 0.0, 0.005, 1000, hub.make_opts(tol=1e-10), v)
    # obs[n, k] = (t, norm, E/N_s, d) of member k at t = n dt; log[n, k, 0] = Krylov dimension m
    B.close()
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhub.so")

HUB_OK = 0
HUB_E_INVALID = -1
HUB_E_SECTOR = -2
HUB_E_NOMEM = -3
HUB_E_DEVICE = -4
HUB_E_NOT_CONVERGED = -5
HUB_E_DEGENERATE = -6
HUB_C128 = 0
HUB_C64 = 1

STATUS_NAMES = {0: "HUB_OK", -1: "HUB_E_INVALID", -2: "HUB_E_SECTOR", -3: "HUB_E_NOMEM",
                -4: "HUB_E_DEVICE", -5: "HUB_E_NOT_CONVERGED", -6: "HUB_E_DEGENERATE"}

# Every symbol include/hub.h declares.
EXPORTS = ("hub_basis_create", "hub_basis_destroy", "hub_basis_info", "hub_basis_states",
           "hub_basis_classes", "hub_basis_hops",
           "hub_apply_H", "hub_observables", "hub_krylov_expm_step", "hub_propagate",
           "hub_ground_state", "hub_pulse_A", "hub_last_error", "hub_profile_enable",
           "hub_profile_read", "hub_apply_cop", "hub_dot", "hub_greens_diag",
           "hub_mlp_forward", "hub_mlp_workspace_bytes", "hub_mlp_train_step", "hub_controller_features",
           "hub_controller_load", "hub_controller_enable", "hub_controller_read_stats",
           "hub_set_apply_path", "hub_spectral", "hub_set_schedule", "hub_observables_noalloc",
           "hub_tune", "hub_set_tuning", "hub_get_plan", "hub_set_greens_path",
           "hub_set_propagate_path")

# Controller MLP sizes (HUB_MLP_* in hub.h).
MLP_IN, MLP_HID, MLP_OUT = 8, 64, 1
MLP_NPARAM = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_OUT * MLP_HID + MLP_OUT


class HubError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class hub_lattice(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32),
                ("bond_i", ctypes.POINTER(ctypes.c_int32)), ("bond_j", ctypes.POINTER(ctypes.c_int32)),
                ("bond_t", ctypes.POINTER(ctypes.c_double)), ("bond_dx", ctypes.POINTER(ctypes.c_double)),
                ("onsite", ctypes.POINTER(ctypes.c_double)), ("U", ctypes.c_double)]


class hub_pulse(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("A0", ctypes.c_double), ("omega", ctypes.c_double),
                ("t0", ctypes.c_double), ("sigma", ctypes.c_double), ("b", ctypes.c_double)]


class hub_krylov_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("m_max", ctypes.c_int32), ("reorth", ctypes.c_int32),
                ("substeps", ctypes.c_int32), ("m_hint", ctypes.c_int32), ("scheme", ctypes.c_int32)]


class hub_step_info(ctypes.Structure):
    _fields_ = [("m_used", ctypes.c_int32), ("substeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("err_est", ctypes.c_double), ("beta_last", ctypes.c_double)]


class hub_greens_member(ctypes.Structure):
    _fields_ = [("site", ctypes.c_int32), ("spin", ctypes.c_int32), ("dagger", ctypes.c_int32),
                ("start_step", ctypes.c_int32)]


class hub_controller_stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("chunks", ctypes.c_int64), ("fallbacks", ctypes.c_int64),
                ("lanczos_launches", ctypes.c_int64), ("iterations", ctypes.c_int64)]


class hub_tuning(ctypes.Structure):
    _fields_ = [("single_two_pass", ctypes.c_int32), ("block_two_pass", ctypes.c_int32 * 4),
                ("apply_group", ctypes.c_int32), ("prop_group", ctypes.c_int32),
                ("apply_us", (ctypes.c_double * 2) * 4), ("step_us", ctypes.c_double * 4),
                ("prop_group_large", ctypes.c_int32), ("step_us_large", ctypes.c_double * 4)]


class hub_obs(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("norm", ctypes.c_double), ("energy_per_site", ctypes.c_double),
                ("docc_per_site", ctypes.c_double)]


_lib_handle = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhub.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(path):
        raise RuntimeError(f"libhub.so not found at {path}: run paper_2005_13498_amd.build first")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "hub_basis_create": ([P(hub_lattice), i32, i32, i32, P(vp)], i32),
        "hub_basis_destroy": ([vp], None),
        "hub_basis_info": ([vp, P(i64), P(i32), P(i32)], i32),
        "hub_basis_states": ([vp, P(ctypes.c_uint32), P(ctypes.c_uint32)], i32),
        "hub_basis_classes": ([vp, P(dbl), P(dbl), P(i32), P(dbl)], i32),
        "hub_basis_hops": ([vp, i32, P(i32), P(i32), P(i32), P(i32), P(i64)], i32),
        "hub_apply_H": ([vp, P(dbl), i32, i32, vp, vp, vp], i32),
        "hub_observables": ([vp, P(dbl), i32, i32, vp, P(hub_obs), P(dbl), vp], i32),
        "hub_observables_noalloc": ([vp, P(dbl), i32, i32, vp, P(hub_obs), P(dbl), vp], i32),
        "hub_krylov_expm_step": ([vp, P(dbl), dbl, P(hub_krylov_opts), i32, i32, vp, P(hub_step_info), vp], i32),
        "hub_propagate": ([vp, P(hub_pulse), dbl, dbl, i32, P(hub_krylov_opts), i32, i32, vp, P(hub_obs),
                           P(hub_step_info), vp], i32),
        "hub_ground_state": ([vp, dbl, P(hub_krylov_opts), vp, P(dbl), P(dbl), vp], i32),
        "hub_pulse_A": ([P(hub_pulse), dbl, P(dbl)], i32),
        "hub_last_error": ([], ctypes.c_char_p),
        "hub_profile_enable": ([vp, i32], i32),
        "hub_profile_read": ([vp, P(i64), P(dbl), P(dbl)], i32),
        "hub_apply_cop": ([vp, vp, i32, i32, i32, i32, i32, vp, vp, vp], i32),
        "hub_dot": ([vp, i32, i32, vp, vp, P(dbl), vp], i32),
        "hub_greens_diag": ([vp, i32, P(vp), P(hub_pulse), dbl, dbl, i32, P(hub_krylov_opts), i32, i32,
                             P(hub_greens_member), vp, P(dbl), vp], i32),
        "hub_mlp_forward": ([i32, vp, i32, vp, vp, vp], i32),
        "hub_mlp_workspace_bytes": ([i32], i64),
        "hub_mlp_train_step": ([i32, vp, vp, vp, i32, ctypes.c_float, i32, vp, vp, vp, vp, vp], i32),
        "hub_controller_features": ([P(hub_pulse), dbl, dbl, i32, dbl, P(hub_krylov_opts), P(hub_step_info), i32,
                                     P(ctypes.c_float), P(ctypes.c_float)], i32),
        "hub_controller_load": ([vp, P(ctypes.c_float), i32], i32),
        "hub_controller_enable": ([vp, i32, i32, i32], i32),
        "hub_controller_read_stats": ([vp, P(hub_controller_stats)], i32),
        "hub_set_apply_path": ([vp, i32], i32),
        "hub_set_greens_path": ([vp, i32], i32),
        "hub_set_propagate_path": ([vp, i32], i32),
        "hub_set_schedule": ([vp, i32, i32], i32),
        "hub_tune": ([vp, i32, i32, P(hub_tuning), vp], i32),
        "hub_set_tuning": ([vp, i32, P(hub_tuning)], i32),
        "hub_get_plan": ([vp, i32, i32, i32, P(i32), P(i32), P(i32)], i32),
        "hub_spectral": ([i32, i32, i32, vp, P(i32), dbl, dbl, i32, vp, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib_handle = lib
    return lib


def _check(status: int, allow=()):
    if status != HUB_OK and status not in allow:
        msg = load_library().hub_last_error()
        raise HubError(status, msg.decode() if msg else "")
    return status


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dbl_array(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def make_lattice(lattice, U: float):
    """hub_lattice from a synth.Lattice (keeps the backing arrays alive)."""
    bi, bj, bt, bdx = lattice.arrays()
    nb = len(bi)
    keep = [(ctypes.c_int32 * max(nb, 1))(*bi), (ctypes.c_int32 * max(nb, 1))(*bj),
            (ctypes.c_double * max(nb, 1))(*bt), (ctypes.c_double * max(nb, 1))(*bdx)]
    onsite = None
    if lattice.onsite is not None:
        onsite = (ctypes.c_double * lattice.n_sites)(*lattice.onsite)
        keep.append(onsite)
    L = hub_lattice(lattice.n_sites, nb, keep[0], keep[1], keep[2], keep[3],
                    ctypes.cast(onsite, ctypes.POINTER(ctypes.c_double)) if onsite is not None else None,
                    float(U))
    return L, keep


def make_pulse(p) -> hub_pulse:
    kind, A0, omega, t0, sigma, b = p.as_tuple() if hasattr(p, "as_tuple") else p
    return hub_pulse(int(kind), float(A0), float(omega), float(t0), float(sigma), float(b))


def make_opts(tol=1e-10, m_max=30, reorth=0, substeps=1, m_hint=0, scheme=0) -> hub_krylov_opts:
    return hub_krylov_opts(float(tol), int(m_max), int(reorth), int(substeps), int(m_hint), int(scheme))


# ------------------------------------------------------------------- ABI calls

def hub_basis_create(lattice, U: float, n_up: int, n_dn: int, device: int = 0) -> int:
    lib = load_library()
    L, keep = make_lattice(lattice, U)
    h = ctypes.c_void_p()
    _check(lib.hub_basis_create(ctypes.byref(L), int(n_up), int(n_dn), int(device), ctypes.byref(h)))
    return h.value


def hub_basis_destroy(h) -> None:
    load_library().hub_basis_destroy(ctypes.c_void_p(h))


def hub_basis_info(h):
    d, du, dd = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().hub_basis_info(ctypes.c_void_p(h), ctypes.byref(d), ctypes.byref(du), ctypes.byref(dd)))
    return d.value, du.value, dd.value


def hub_basis_states(h):
    _, du, dd = hub_basis_info(h)
    up = np.zeros(du, dtype=np.uint32)
    dn = np.zeros(dd, dtype=np.uint32)
    _check(load_library().hub_basis_states(ctypes.c_void_p(h),
                                           up.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                           dn.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return up, dn


def hub_basis_classes(h):
    """(t[nc], d[nc], norm_inf)."""
    t = np.zeros(8)
    d = np.zeros(8)
    nc = ctypes.c_int32()
    ni = ctypes.c_double()
    P = ctypes.POINTER(ctypes.c_double)
    _check(load_library().hub_basis_classes(ctypes.c_void_p(h), t.ctypes.data_as(P), d.ctypes.data_as(P),
                                            ctypes.byref(nc), ctypes.byref(ni)))
    return t[: nc.value], d[: nc.value], ni.value


def hub_basis_hops(h, spin: int):
    """(ptr[dim_spin+1], src, sign, cls) of the gather-form hop table."""
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.hub_basis_hops(ctypes.c_void_p(h), int(spin), None, None, None, None, ctypes.byref(n)))
    _, du, dd = hub_basis_info(h)
    ptr = np.zeros((du if spin == 0 else dd) + 1, dtype=np.int32)
    src = np.zeros(max(n.value, 1), dtype=np.int32)
    sgn = np.zeros(max(n.value, 1), dtype=np.int32)
    cls = np.zeros(max(n.value, 1), dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    _check(lib.hub_basis_hops(ctypes.c_void_p(h), int(spin), ptr.ctypes.data_as(P), src.ctypes.data_as(P),
                              sgn.ctypes.data_as(P), cls.ctypes.data_as(P), ctypes.byref(n)))
    k = n.value
    return ptr, src[:k], sgn[:k], cls[:k]


def _prec_of(t):
    import torch
    if t.dtype == torch.complex128:
        return HUB_C128
    if t.dtype == torch.complex64:
        return HUB_C64
    raise TypeError("device vectors must be complex128 or complex64 tensors")


def hub_apply_H(h, A: Sequence[float], x, y, stream=None) -> None:
    """y = H(A_k) x_k for the nvec = len(A) vectors stored in x (contiguous)."""
    A = list(np.atleast_1d(A))
    assert x.is_contiguous() and y.is_contiguous() and x.dtype == y.dtype
    _check(load_library().hub_apply_H(ctypes.c_void_p(h), _dbl_array(A), _prec_of(x), len(A), _dptr(x), _dptr(y),
                                      _stream_ptr(stream)))


def hub_observables(h, A: Sequence[float], v, site=False, stream=None, noalloc=False):
    """(obs array [nvec, 4] = t, norm, energy/site, docc/site; site docc or None).
    noalloc: call hub_observables_noalloc (no device allocation)."""
    A = list(np.atleast_1d(A))
    n = len(A)
    out = (hub_obs * n)()
    sd = np.zeros(n * _n_sites_cache.get(h, 16), dtype=np.float64) if site else None
    lib = load_library()
    fn = lib.hub_observables_noalloc if noalloc else lib.hub_observables
    _check(fn(ctypes.c_void_p(h), _dbl_array(A), _prec_of(v), n, _dptr(v), out,
              sd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if site else None, _stream_ptr(stream)))
    arr = np.array([[o.t, o.norm, o.energy_per_site, o.docc_per_site] for o in out])
    if site:
        ns = _n_sites_cache.get(h, 16)
        return arr, sd.reshape(n, ns)
    return arr, None


_n_sites_cache = {}


_INFO_DTYPE = np.dtype([("m_used", np.int32), ("substeps", np.int32), ("converged", np.int32),
                        ("breakdown", np.int32), ("err_est", np.float64), ("beta_last", np.float64)])


def _info_array(info, n):
    """[n, 6] float array (m_used, substeps, converged, breakdown, err_est,
    beta_last) read straight from the ctypes buffer."""
    rec = np.frombuffer(info, dtype=_INFO_DTYPE, count=n)
    return np.stack([rec[f].astype(np.float64) for f in _INFO_DTYPE.names], axis=1)


def hub_krylov_expm_step(h, A_mid: Sequence[float], dt: float, opts: hub_krylov_opts, v, stream=None,
                         allow_not_converged=False):
    A = list(np.atleast_1d(A_mid))
    info = (hub_step_info * len(A))()
    st = _check(load_library().hub_krylov_expm_step(ctypes.c_void_p(h), _dbl_array(A), float(dt),
                                                    ctypes.byref(opts), _prec_of(v), len(A), _dptr(v), info,
                                                    _stream_ptr(stream)),
                allow=(HUB_E_NOT_CONVERGED,) if allow_not_converged else ())
    return st, _info_array(info, len(A))


def hub_propagate(h, pulses, t_start: float, dt: float, n_steps: int, opts: hub_krylov_opts, v,
                  want_obs=True, want_log=True, stream=None, allow_not_converged=False):
    """Returns (status, obs [n_steps+1, nvec, 4] or None, log [n_steps, nvec, 6] or None)."""
    pulses = list(pulses)
    nvec = len(pulses)
    parr = (hub_pulse * nvec)(*[make_pulse(p) for p in pulses])
    obs = (hub_obs * ((n_steps + 1) * nvec))() if want_obs else None
    log = (hub_step_info * max(1, n_steps * nvec))() if want_log else None
    st = _check(load_library().hub_propagate(ctypes.c_void_p(h), parr, float(t_start), float(dt), int(n_steps),
                                             ctypes.byref(opts), _prec_of(v), nvec, _dptr(v), obs, log,
                                             _stream_ptr(stream)),
                allow=(HUB_E_NOT_CONVERGED,) if allow_not_converged else ())
    o = None
    if want_obs:
        o = np.frombuffer(obs, dtype=np.float64).reshape(n_steps + 1, nvec, 4).copy()
    lg = _info_array(log, n_steps * nvec).reshape(n_steps, nvec, 6) if (want_log and n_steps > 0) else None
    return st, o, lg


def hub_ground_state(h, A: float, v_out, opts: Optional[hub_krylov_opts] = None, stream=None,
                     allow_degenerate=False):
    E0, gap = ctypes.c_double(), ctypes.c_double()
    st = _check(load_library().hub_ground_state(ctypes.c_void_p(h), float(A),
                                                ctypes.byref(opts) if opts is not None else None,
                                                _dptr(v_out), ctypes.byref(E0), ctypes.byref(gap),
                                                _stream_ptr(stream)),
                allow=(HUB_E_DEGENERATE,) if allow_degenerate else ())
    return st, E0.value, gap.value


def hub_pulse_A(pulse, t: float) -> float:
    A = ctypes.c_double()
    p = make_pulse(pulse)
    _check(load_library().hub_pulse_A(ctypes.byref(p), float(t), ctypes.byref(A)))
    return A.value


def hub_profile_enable(h, on) -> None:
    """False/0 off; True/1 time every eligible H*v; k > 1 every k-th."""
    k = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _check(load_library().hub_profile_enable(ctypes.c_void_p(h), k))


def hub_profile_read(h):
    n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().hub_profile_read(ctypes.c_void_p(h), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)))
    return n.value, ms.value, b.value


def hub_apply_cop(h_from, h_to, site: int, spin: int, dagger: bool, x, y, nvec: int = 1, stream=None) -> None:
    """y = c_{site,spin} x (dagger False) or c^dag x, from h_from's sector to h_to's."""
    _check(load_library().hub_apply_cop(ctypes.c_void_p(h_from), ctypes.c_void_p(h_to), int(site), int(spin),
                                        1 if dagger else 0, _prec_of(x), int(nvec), _dptr(x), _dptr(y),
                                        _stream_ptr(stream)))


def hub_dot(h, x, y, nvec: int = 1, stream=None) -> np.ndarray:
    """<x_k|y_k> for nvec pairs (complex array)."""
    out = np.zeros(2 * nvec)
    _check(load_library().hub_dot(ctypes.c_void_p(h), _prec_of(x), int(nvec), _dptr(x), _dptr(y),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream)))
    return out[0::2] + 1j * out[1::2]


def hub_greens_diag(h, targets, pulse, t_start: float, dt: float, n_rel: int, opts, members, psi, stream=None):
    """Overlaps o[k, s] (complex) of the members (site, spin, dagger, start_step)."""
    nt = len(targets)
    tarr = (ctypes.c_void_p * nt)(*[ctypes.c_void_p(t) for t in targets])
    nm = len(members)
    marr = (hub_greens_member * nm)(*[hub_greens_member(*[int(v) for v in m]) for m in members])
    out = np.zeros(nm * (n_rel + 1) * 2)
    p = make_pulse(pulse)
    _check(load_library().hub_greens_diag(ctypes.c_void_p(h), nt, tarr, ctypes.byref(p), float(t_start), float(dt),
                                          int(n_rel), ctypes.byref(opts), _prec_of(psi), nm, marr, _dptr(psi),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream)))
    o = out.reshape(nm, n_rel + 1, 2)
    return o[..., 0] + 1j * o[..., 1]


def _device_of(t) -> int:
    return t.device.index if t.device.index is not None else 0


def hub_mlp_forward(params, feats, out, stream=None) -> None:
    """out[r, 0] = MLP(feats[r, :8]); float32 device tensors."""
    _check(load_library().hub_mlp_forward(_device_of(params), _dptr(params), int(feats.shape[0]), _dptr(feats),
                                          _dptr(out), _stream_ptr(stream)))


def hub_mlp_workspace_bytes(n_rows: int) -> int:
    return int(load_library().hub_mlp_workspace_bytes(int(n_rows)))


def hub_mlp_train_step(params, adam_m, adam_v, t: int, lr: float, feats, targets, loss, workspace,
                       stream=None) -> None:
    """One Adam step on the mean squared error (all float32 device tensors)."""
    _check(load_library().hub_mlp_train_step(_device_of(params), _dptr(params), _dptr(adam_m), _dptr(adam_v),
                                             int(t), float(lr), int(feats.shape[0]), _dptr(feats), _dptr(targets),
                                             _dptr(loss), _dptr(workspace), _stream_ptr(stream)))


def hub_controller_features(pulse, t_start: float, dt: float, norm_inf: float, opts, log_rows, chunk: int):
    """Training rows (feats [n, 8], targets [n, 2]) from one vector's step log.

    log_rows: array [n_steps, 6] as returned in hub_propagate's log for one
    vector (m_used, substeps, converged, breakdown, err_est, beta_last)."""
    lr = np.asarray(log_rows)
    n = lr.shape[0]
    info = (hub_step_info * max(1, n))()
    for k in range(n):
        info[k] = hub_step_info(int(lr[k, 0]), int(lr[k, 1]), int(lr[k, 2]), int(lr[k, 3]), float(lr[k, 4]),
                                float(lr[k, 5]))
    feats = np.zeros((max(1, n), MLP_IN), dtype=np.float32)
    targ = np.zeros((max(1, n), MLP_OUT), dtype=np.float32)
    p = make_pulse(pulse)
    Pf = ctypes.POINTER(ctypes.c_float)
    _check(load_library().hub_controller_features(ctypes.byref(p), float(t_start), float(dt), n, float(norm_inf),
                                                  ctypes.byref(opts), info, int(chunk), feats.ctypes.data_as(Pf),
                                                  targ.ctypes.data_as(Pf)))
    return feats[:n], targ[:n]


def hub_controller_load(h, params) -> None:
    arr = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
    _check(load_library().hub_controller_load(ctypes.c_void_p(h), arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                              int(arr.size)))


def hub_controller_enable(h, on: bool, chunk: int = 16, margin: int = 1) -> None:
    _check(load_library().hub_controller_enable(ctypes.c_void_p(h), 1 if on else 0, int(chunk), int(margin)))


def hub_controller_read_stats(h) -> dict:
    s = hub_controller_stats()
    _check(load_library().hub_controller_read_stats(ctypes.c_void_p(h), ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in hub_controller_stats._fields_}


def hub_spectral(overlaps, lesser, dt: float, eps: float, nu, out, stream=None) -> None:
    """A[m, f] from overlaps [n_members, n_s] (complex128 device tensor), nu
    [n_nu] and out [n_members, n_nu] (float64 device tensors); lesser: host
    sequence of flags (1 removal / c, 0 addition / c^dag)."""
    nm, ns = int(overlaps.shape[0]), int(overlaps.shape[1])
    flags = (ctypes.c_int32 * max(1, nm))(*[int(bool(x)) for x in lesser])
    _check(load_library().hub_spectral(_device_of(overlaps), nm, ns, _dptr(overlaps), flags, float(dt), float(eps),
                                       int(nu.shape[0]), _dptr(nu), _dptr(out), _stream_ptr(stream)))


def hub_set_apply_path(h, path: int) -> None:
    """-1 automatic, 0 one-pass, 1 two-pass H*v kernels for single vectors."""
    _check(load_library().hub_set_apply_path(ctypes.c_void_p(h), int(path)))


def hub_set_greens_path(h, path: int) -> None:
    """hub_greens_diag's member stepper: -1 automatic, 0 per-sector batches,
    1 the persistent one-launch member stepper."""
    _check(load_library().hub_set_greens_path(ctypes.c_void_p(h), int(path)))


def hub_set_propagate_path(h, path: int) -> None:
    """hub_propagate's path: -1 automatic, 0 launches per Lanczos iteration,
    1 the resident one-launch stepper (small sectors)."""
    _check(load_library().hub_set_propagate_path(ctypes.c_void_p(h), int(path)))


def hub_set_schedule(h, chunk: int, margin: int = 1) -> None:
    """Default propagation schedule: chunks of `chunk` steps without host
    synchronisation (0: one synchronisation per step)."""
    _check(load_library().hub_set_schedule(ctypes.c_void_p(h), int(chunk), int(margin)))


def tuning_to_dict(t: hub_tuning) -> dict:
    return {"single_two_pass": t.single_two_pass, "block_two_pass": list(t.block_two_pass),
            "apply_group": t.apply_group, "prop_group": t.prop_group,
            "apply_us": [list(r) for r in t.apply_us], "step_us": list(t.step_us),
            "prop_group_large": t.prop_group_large, "step_us_large": list(t.step_us_large)}


def tuning_from_dict(d: dict) -> hub_tuning:
    t = hub_tuning()
    t.single_two_pass = int(d["single_two_pass"])
    for k in range(4):
        t.block_two_pass[k] = int(d["block_two_pass"][k])
        t.step_us[k] = float(d.get("step_us", [0.0] * 4)[k])
        t.step_us_large[k] = float(d.get("step_us_large", [0.0] * 4)[k])
        for p in range(2):
            t.apply_us[k][p] = float(d.get("apply_us", [[0.0, 0.0]] * 4)[k][p])
    t.apply_group = int(d["apply_group"])
    t.prop_group = int(d["prop_group"])
    t.prop_group_large = int(d.get("prop_group_large", d["prop_group"]))  # tables from before the large batch
    return t


def hub_tune(h, prec: int, reps: int = 10, stream=None) -> dict:
    """Measure and install the kernel plan of one precision; returns it as a dict."""
    t = hub_tuning()
    _check(load_library().hub_tune(ctypes.c_void_p(h), int(prec), int(reps), ctypes.byref(t), _stream_ptr(stream)))
    return tuning_to_dict(t)


def hub_set_tuning(h, prec: int, table) -> None:
    """Install a plan (dict from hub_tune), or the built-in rules with None."""
    t = tuning_from_dict(table) if table is not None else None
    _check(load_library().hub_set_tuning(ctypes.c_void_p(h), int(prec), ctypes.byref(t) if t is not None else None))


def hub_get_plan(h, prec: int, nvec: int, propagate: bool = True):
    """[(group size, kernels)] with kernels 0 one pass, 1 two-pass single, 2 two-pass block."""
    n = ctypes.c_int32()
    sizes = (ctypes.c_int32 * max(1, nvec))()
    kern = (ctypes.c_int32 * max(1, nvec))()
    _check(load_library().hub_get_plan(ctypes.c_void_p(h), int(prec), int(nvec), 1 if propagate else 0,
                                       ctypes.byref(n), sizes, kern))
    return [(sizes[k], kern[k]) for k in range(n.value)]


class Basis:
    """Owning wrapper of a basis handle."""

    def __init__(self, lattice, U: float, n_up: int, n_dn: int, device: int = 0):
        self.lattice = lattice
        self.U = U
        self.handle = hub_basis_create(lattice, U, n_up, n_dn, device)
        self.dim, self.dim_up, self.dim_dn = hub_basis_info(self.handle)
        self.n_sites = lattice.n_sites
        _n_sites_cache[self.handle] = lattice.n_sites

    def close(self):
        if self.handle:
            hub_basis_destroy(self.handle)
            _n_sites_cache.pop(self.handle, None)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
