"""MI355X-native boundary-MPS contraction and sampling of 2D tensor-network states.

Thin Python binding of the C ABI in ``include/tn.h`` (``libtnbmps.so``, built
in this directory by ``build_lib.py``).  This module only marshals arguments:
PyTorch supplies device memory and the HIP stream, and every step of the
computation runs in the library's HIP kernels.  There is no CPU fallback: if
the library or a GPU is missing, the calls raise.

Operations (Rudolph & Tindall, "Simulating and Sampling from Quantum Circuits
with 2D Tensor Networks"):

* ``boundary_contract`` -- norm <psi|psi> by boundary MPSs and the one-site fit;
* ``environments``      -- one-site density matrices and nearest-neighbour <ZZ>;
* ``sample``            -- sequential bitstring sampling with q(x) and p(x).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnbmps.so")

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
STATUS = {0: "TN_OK", 1: "TN_ERR_INVALID", 2: "TN_ERR_SHAPE", 3: "TN_ERR_OOM", 4: "TN_ERR_HIP",
          5: "TN_ERR_NUMERIC", 6: "TN_ERR_UNSUPPORTED"}

# every symbol declared in include/tn.h
EXPORTS = ["tn_default_opts", "tn_create", "tn_destroy", "tn_boundary_contract", "tn_environments",
           "tn_sample", "tn_amplitude", "tn_sample_stats", "tn_last_error", "tn_get_counters", "tn_set_timing",
           "tn_set_autotune", "tn_plan_report", "tn_test_contract", "tn_test_qr", "tn_test_svd", "tn_test_set_mask",
           "tn_test_sample_config", "tn_sample_stats_noalloc", "tn_bp", "tn_test_eig", "tn_simple_update"]


class TnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class c_peps(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("phys", ctypes.POINTER(ctypes.c_int32)), ("dim_h", ctypes.POINTER(ctypes.c_int32)),
                ("dim_v", ctypes.POINTER(ctypes.c_int32)), ("site_index", ctypes.POINTER(ctypes.c_int32)),
                ("dtype", ctypes.c_int), ("site", ctypes.POINTER(ctypes.c_void_p))]


class c_opts(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_int32), ("chi_x", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("init", ctypes.c_int32), ("prec", ctypes.c_int),
                ("init_seed", ctypes.c_uint64), ("workspace_cap", ctypes.c_size_t),
                ("svd_cutoff", ctypes.c_double), ("chi_x_min", ctypes.c_int32)]


_lib = None


def lib(path: Optional[str] = None):
    """Loads the C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: build it with `python -m paper_2507_11424_amd.build_lib`")
    L = ctypes.CDLL(p)
    vp, i32, i64, u64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
    L.tn_default_opts.argtypes = [ctypes.POINTER(c_opts)]
    L.tn_default_opts.restype = None
    L.tn_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    L.tn_destroy.argtypes = [vp]
    L.tn_boundary_contract.argtypes = [vp, ctypes.POINTER(c_peps), ctypes.POINTER(c_opts), dp, dp]
    L.tn_environments.argtypes = [vp, ctypes.POINTER(c_peps), ctypes.POINTER(c_opts), vp, vp, vp, vp, vp]
    L.tn_sample.argtypes = [vp, ctypes.POINTER(c_peps), ctypes.POINTER(c_opts), u64, u64, i64, vp, vp, vp, vp, vp]
    L.tn_amplitude.argtypes = [vp, ctypes.POINTER(c_peps), ctypes.POINTER(c_opts), u64, i64, vp, vp, vp]
    L.tn_sample_stats.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp, ctypes.c_double, vp, vp]
    L.tn_sample_stats_noalloc.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp, ctypes.c_double, vp, vp]
    L.tn_last_error.argtypes = [vp]
    L.tn_last_error.restype = ctypes.c_char_p
    L.tn_get_counters.argtypes = [vp, dp, ctypes.POINTER(i64), dp, dp, ctypes.POINTER(i64), dp,
                                  ctypes.POINTER(i64), dp, dp, ctypes.POINTER(i64)]
    L.tn_set_timing.argtypes = [vp, ctypes.c_int]
    L.tn_set_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_char_p]
    L.tn_plan_report.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    L.tn_plan_report.restype = ctypes.c_int
    L.tn_test_contract.argtypes = [vp, ctypes.c_int, ctypes.c_char_p, vp, ctypes.POINTER(i32), ctypes.c_int,
                                   ctypes.c_char_p, vp, ctypes.POINTER(i32), ctypes.c_int,
                                   ctypes.c_char_p, vp, ctypes.POINTER(i32), ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int]
    L.tn_test_qr.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_int]
    L.tn_test_svd.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_double, ctypes.c_int, vp, vp,
                              ctypes.c_int, vp]
    L.tn_test_set_mask.argtypes = [vp, vp, ctypes.c_char]
    L.tn_test_sample_config.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]
    ip = ctypes.POINTER(ctypes.c_int)
    L.tn_bp.argtypes = [vp, ctypes.POINTER(c_peps), ctypes.c_int, ctypes.c_double, dp, dp, ip, dp, dp, dp,
                        ctypes.c_int, ip, vp]
    L.tn_test_eig.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
    L.tn_simple_update.argtypes = [vp, ctypes.POINTER(c_peps), vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, vp, dp, vp, vp]
    for f in ("tn_create", "tn_destroy", "tn_boundary_contract", "tn_environments", "tn_sample",
              "tn_get_counters", "tn_set_timing", "tn_set_autotune", "tn_test_contract",
              "tn_test_qr", "tn_test_svd", "tn_test_set_mask", "tn_amplitude", "tn_sample_stats",
              "tn_test_sample_config", "tn_sample_stats_noalloc", "tn_bp", "tn_test_eig", "tn_simple_update"):
        getattr(L, f).restype = ctypes.c_int
    if path is None:
        _lib = L
    return L


def _i32(a) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
    return (ctypes.c_int32 * max(len(a), 1))(*a.tolist())


def make_opts(chi=16, chi_x=None, sweeps=2, direction=0, force_fit=False, prec="fp64", init_seed=0,
              workspace_cap=0, svd_cutoff=0.0, chi_x_min=1) -> c_opts:
    o = c_opts()
    lib().tn_default_opts(ctypes.byref(o))
    o.chi = int(chi)
    o.chi_x = int(chi if chi_x is None else chi_x)
    o.sweeps = int(sweeps)
    o.direction = int(direction)
    o.init = 1 if force_fit else 0
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.init_seed = int(init_seed)
    o.workspace_cap = int(workspace_cap)
    o.svd_cutoff = float(svd_cutoff)
    o.chi_x_min = int(chi_x_min)
    return o


class Peps:
    """A PEPS on the device: lattice arrays (host) + one device tensor per site,
    index order [p][u][l][d][r], complex128 or complex64 torch tensors."""

    def __init__(self, lattice, site_tensors: Sequence):
        import torch
        self.lattice = lattice
        self.tensors = list(site_tensors)  # keeps the device memory alive
        dt = self.tensors[0].dtype
        if dt not in (torch.complex128, torch.complex64):
            raise TypeError("site tensors must be complex128 or complex64")
        if any(t.dtype != dt for t in self.tensors):
            raise TypeError("all site tensors must share one dtype")
        self.dtype = dt
        self._phys = _i32(lattice.phys)
        self._dh = _i32(lattice.dim_h)
        self._dv = _i32(lattice.dim_v)
        self._si = _i32(lattice.site_index)
        n = lattice.rows * lattice.cols
        if len(self.tensors) != n:
            raise ValueError("one tensor per grid position expected")
        self._ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.tensors])
        self.c = c_peps(lattice.rows, lattice.cols, self._phys, self._dh, self._dv, self._si,
                        0 if dt == torch.complex128 else 1, self._ptrs)

    @property
    def n_qubits(self) -> int:
        return int(self.lattice.n_qubits)

    @staticmethod
    def from_numpy(lattice, tensors, dtype="c128", device="cuda"):
        """Copies host arrays ([rows][cols] nested list or flat list) to the device."""
        import torch
        flat = [t for row in tensors for t in row] if isinstance(tensors[0], (list, tuple)) else list(tensors)
        td = torch.complex128 if dtype == "c128" else torch.complex64
        dev = [torch.from_numpy(np.ascontiguousarray(t)).to(device=device, dtype=td) for t in flat]
        return Peps(lattice, dev)


class Handle:
    """Library handle bound to a device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib().tn_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise TnError(st, "tn_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().tn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise TnError(st, lib().tn_last_error(self.h).decode())

    # ---------------------------------------------------------------- operations
    def boundary_contract(self, peps: Peps, opts: c_opts):
        la, ar = ctypes.c_double(), ctypes.c_double()
        self._check(lib().tn_boundary_contract(self.h, ctypes.byref(peps.c), ctypes.byref(opts),
                                               ctypes.byref(la), ctypes.byref(ar)))
        return la.value, ar.value

    def environments(self, peps: Peps, opts: c_opts, want_zz: bool = True, want_p2: bool = True):
        import torch
        L = peps.lattice
        dev = peps.tensors[0].device
        f64 = dict(dtype=torch.float64, device=dev)
        rho = torch.empty((L.rows * L.cols, 2, 2, 2), **f64)
        zzh = torch.empty((L.rows, max(L.cols - 1, 0)), **f64) if want_zz else None
        zzv = torch.empty((max(L.rows - 1, 0), L.cols), **f64) if want_zz else None
        p2h = torch.empty((L.rows, max(L.cols - 1, 0), 4), **f64) if want_p2 else None
        p2v = torch.empty((max(L.rows - 1, 0), L.cols, 4), **f64) if want_p2 else None
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None  # noqa: E731
        self._check(lib().tn_environments(self.h, ctypes.byref(peps.c), ctypes.byref(opts), ptr(rho), ptr(zzh),
                                          ptr(zzv), ptr(p2h), ptr(p2v)))
        rho1 = torch.view_as_complex(rho).reshape(L.rows, L.cols, 2, 2)
        return dict(rho1=rho1, zz_h=zzh, zz_v=zzv, p2_h=p2h, p2_v=p2v)

    def sample(self, peps: Peps, opts: c_opts, n: int, seed: int = 0, first: int = 0, uniforms=None,
               want_logp: bool = True, want_chi: bool = False):
        """bits [n][N] uint8, log q [n], log p [n] (or None); with want_chi also
        the per-row amplitude-boundary bonds [n][rows] int32 (see tn_sample)."""
        import torch
        dev = peps.tensors[0].device
        nq = peps.n_qubits
        bits = torch.empty((n, nq), dtype=torch.uint8, device=dev)
        lq = torch.empty((n,), dtype=torch.float64, device=dev)
        lp = torch.empty((n,), dtype=torch.float64, device=dev) if want_logp else None
        if uniforms is not None:
            uniforms = uniforms.to(device=dev, dtype=torch.float64).contiguous()
            if tuple(uniforms.shape) != (n, nq):
                raise ValueError("uniforms must have shape [n][N]")
        up = ctypes.c_void_p(uniforms.data_ptr()) if uniforms is not None else None
        cu = torch.empty((n, peps.c.rows), dtype=torch.int32, device=dev) if want_chi else None
        self._check(lib().tn_sample(self.h, ctypes.byref(peps.c), ctypes.byref(opts), seed, first, n, up,
                                    ctypes.c_void_p(bits.data_ptr()), ctypes.c_void_p(lq.data_ptr()),
                                    ctypes.c_void_p(lp.data_ptr()) if lp is not None else None,
                                    ctypes.c_void_p(cu.data_ptr()) if cu is not None else None))
        return (bits, lq, lp, cu) if want_chi else (bits, lq, lp)

    def amplitude(self, peps: Peps, opts: c_opts, bits, first: int = 0, want_arg: bool = False):
        """log p(x) = 2 log|<x|psi>| (and arg <x|psi>) for bitstrings bits [n][N]
        by a separate contraction with bond opts.chi_x (see tn_amplitude)."""
        import torch
        dev = peps.tensors[0].device
        bits = bits.to(device=dev, dtype=torch.uint8).contiguous()
        if bits.dim() != 2 or bits.shape[1] != peps.n_qubits:
            raise ValueError("bits must have shape [n][N]")
        n = bits.shape[0]
        lp = torch.empty((n,), dtype=torch.float64, device=dev)
        ar = torch.empty((n,), dtype=torch.float64, device=dev) if want_arg else None
        self._check(lib().tn_amplitude(self.h, ctypes.byref(peps.c), ctypes.byref(opts), first, n,
                                       ctypes.c_void_p(bits.data_ptr()), ctypes.c_void_p(lp.data_ptr()),
                                       ctypes.c_void_p(ar.data_ptr()) if ar is not None else None))
        return (lp, ar) if want_arg else lp

    def sample_stats(self, log_q, log_p, log_Z: float, bits=None):
        """Norm estimate, sample KLD, effective sample size and (with bits) the
        importance-sampled <Z_q> (see tn_sample_stats)."""
        import torch
        dev = log_q.device
        lq = log_q.to(dtype=torch.float64).contiguous()
        lp = log_p.to(device=dev, dtype=torch.float64).contiguous()
        if lq.shape != lp.shape or lq.dim() != 1:
            raise ValueError("log_q and log_p must be 1-d of equal length")
        n = lq.shape[0]
        out = (ctypes.c_double * 3)()
        zis = None
        bp = None
        nq = 0
        if bits is not None:
            bits = bits.to(device=dev, dtype=torch.uint8).contiguous()
            if bits.dim() != 2 or bits.shape[0] != n:
                raise ValueError("bits must have shape [n][N]")
            nq = bits.shape[1]
            zis = torch.empty((nq,), dtype=torch.float64, device=dev)
            bp = ctypes.c_void_p(bits.data_ptr())
        self._check(lib().tn_sample_stats(self.h, n, nq, bp, ctypes.c_void_p(lq.data_ptr()),
                                          ctypes.c_void_p(lp.data_ptr()), float(log_Z), out,
                                          ctypes.c_void_p(zis.data_ptr()) if zis is not None else None))
        res = dict(log_norm_est=out[0], kld=out[1], ess=out[2])
        if zis is not None:
            res["z_is"] = zis
        return res

    def bp(self, peps: Peps, max_sweeps: int = 1000, tol: float = 1e-13, loops: bool = True,
           want_messages: bool = False):
        """Belief propagation on the norm network: log|Z_BP|, arg Z_BP, sweeps,
        last change and (with loops) the loop BP error eps with its per-loop
        values; with want_messages also the final messages [N][4][Dm][Dm]
        (see tn_bp)."""
        import torch
        la, ar, ch, em = (ctypes.c_double() for _ in range(4))
        sw, nl = ctypes.c_int(), ctypes.c_int()
        L = peps.lattice
        cap = max(1, (L.rows - 1) * (L.cols - 1))
        eps = (ctypes.c_double * cap)()
        msgs = None
        if want_messages:
            dm = int(max(1, np.max(L.dim_h) if L.dim_h.size else 1, np.max(L.dim_v) if L.dim_v.size else 1))
            msgs = torch.empty((L.rows * L.cols, 4, dm, dm), dtype=torch.complex128, device=peps.tensors[0].device)
        self._check(lib().tn_bp(self.h, ctypes.byref(peps.c), int(max_sweeps), float(tol), ctypes.byref(la),
                                ctypes.byref(ar), ctypes.byref(sw), ctypes.byref(ch),
                                ctypes.byref(em) if loops else None, eps if loops else None, cap,
                                ctypes.byref(nl) if loops else None,
                                ctypes.c_void_p(msgs.data_ptr()) if msgs is not None else None))
        res = dict(log_abs_Z=la.value, arg_Z=ar.value, sweeps=sw.value, last_change=ch.value)
        if loops:
            res["eps"] = em.value
            res["eps_loops"] = np.array(eps[:nl.value])
        if msgs is not None:
            res["messages"] = msgs
        return res

    def simple_update(self, peps: Peps, gates, G, bp_max_sweeps: int = 1000, bp_tol: float = 1e-13,
                      in_place: bool = False, messages_in=None, messages_out=None):
        """Applies two-qubit gates by BP-gauged simple update (see
        tn_simple_update).  gates: sequence of (group, r, c, r2, c2); G: one
        4 x 4 complex matrix for all gates or one per gate.  Returns (Peps of
        the result, gate errors eps (numpy), fidelity estimate prod(1 - eps));
        in_place writes the result into peps's own tensors.  messages_in /
        messages_out: optional complex128 device tensors [rows*cols][4][Dm][Dm]
        (see message_buffer) to start the BP from and to receive the last
        group's messages."""
        import torch
        gl = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 5))
        Gm = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
        stride = 0 if Gm.ndim == 2 else 16
        if Gm.shape[-2:] != (4, 4) or (stride and Gm.shape[0] != gl.shape[0]):
            raise ValueError("G: one 4 x 4 matrix, or one per gate")
        out = peps if in_place else Peps(peps.lattice, [torch.empty_like(t) for t in peps.tensors])
        ptrs = (ctypes.c_void_p * len(out.tensors))(*[t.data_ptr() for t in out.tensors])
        eps = np.zeros(gl.shape[0], dtype=np.float64)
        f = ctypes.c_double()
        self._check(lib().tn_simple_update(self.h, ctypes.byref(peps.c), ptrs, int(gl.shape[0]),
                                           gl.ctypes.data_as(ctypes.c_void_p), Gm.ctypes.data_as(ctypes.c_void_p),
                                           stride, int(bp_max_sweeps), float(bp_tol),
                                           eps.ctypes.data_as(ctypes.c_void_p), ctypes.byref(f),
                                           self._msg_ptr(peps, messages_in), self._msg_ptr(peps, messages_out)))
        return out, eps, f.value

    @staticmethod
    def message_buffer(peps: Peps):
        """A complex128 device tensor [rows*cols][4][Dm][Dm] for BP messages."""
        import torch
        L = peps.lattice
        dm = int(max(1, np.max(L.dim_h) if L.dim_h.size else 1, np.max(L.dim_v) if L.dim_v.size else 1))
        return torch.zeros((L.rows * L.cols, 4, dm, dm), dtype=torch.complex128, device=peps.tensors[0].device)

    @staticmethod
    def _msg_ptr(peps: Peps, m):
        import torch
        if m is None:
            return None
        L = peps.lattice
        dm = int(max(1, np.max(L.dim_h) if L.dim_h.size else 1, np.max(L.dim_v) if L.dim_v.size else 1))
        if (m.dtype != torch.complex128 or tuple(m.shape) != (L.rows * L.cols, 4, dm, dm) or not m.is_contiguous()
                or m.device != peps.tensors[0].device):
            raise ValueError("messages: contiguous complex128 [rows*cols][4][Dm][Dm] on the state's device")
        return ctypes.c_void_p(m.data_ptr())

    def test_eig(self, A):
        """Eigenvalues (unordered), eps and info of complex128 matrices A
        [batch][n][n] by the loop-error eigenvalue kernel (see tn_test_eig)."""
        import torch
        A = A.to(torch.complex128).contiguous()
        batch, n = A.shape[0], A.shape[1]
        lam = torch.empty((batch, n), dtype=torch.complex128, device=A.device)
        eps = torch.empty((batch,), dtype=torch.float64, device=A.device)
        info = torch.empty((batch,), dtype=torch.int32, device=A.device)
        self._check(lib().tn_test_eig(self.h, n, batch, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                      ctypes.c_void_p(eps.data_ptr()), ctypes.c_void_p(info.data_ptr())))
        return lam, eps, info

    def sample_stats_noalloc(self, log_q, log_p, log_Z: float, bits=None, out=None, z_is=None):
        """As sample_stats through tn_sample_stats_noalloc: the library allocates
        nothing (partials in its fixed scratch); `out` (device float64 [3]) and
        `z_is` (device float64 [N], with bits) are the caller's buffers, made
        here if not given.  Asynchronous: returns the device tensors."""
        import torch
        dev = log_q.device
        if log_q.dtype != torch.float64 or log_p.dtype != torch.float64 or not log_q.is_contiguous() \
                or not log_p.is_contiguous() or log_p.device != dev:
            raise ValueError("log_q and log_p must be contiguous float64 tensors on one device")
        if log_q.shape != log_p.shape or log_q.dim() != 1:
            raise ValueError("log_q and log_p must be 1-d of equal length")
        n = log_q.shape[0]
        if out is None:
            out = torch.empty((3,), dtype=torch.float64, device=dev)
        bp = None
        nq = 0
        if bits is not None:
            if bits.dtype != torch.uint8 or not bits.is_contiguous() or bits.dim() != 2 or bits.shape[0] != n:
                raise ValueError("bits must be a contiguous uint8 tensor of shape [n][N]")
            nq = bits.shape[1]
            if z_is is None:
                z_is = torch.empty((nq,), dtype=torch.float64, device=dev)
            bp = ctypes.c_void_p(bits.data_ptr())
        else:
            z_is = None
        self._check(lib().tn_sample_stats_noalloc(self.h, n, nq, bp, ctypes.c_void_p(log_q.data_ptr()),
                                                  ctypes.c_void_p(log_p.data_ptr()), float(log_Z),
                                                  ctypes.c_void_p(out.data_ptr()),
                                                  ctypes.c_void_p(z_is.data_ptr()) if z_is is not None else None))
        return out, z_is

    def counters(self):
        f, ms, qms, qf, mms, gb = (ctypes.c_double() for _ in range(6))
        n, qn, mn, gl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().tn_get_counters(self.h, ctypes.byref(f), ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(qms), ctypes.byref(qn), ctypes.byref(qf),
                                          ctypes.byref(mn), ctypes.byref(mms), ctypes.byref(gb),
                                          ctypes.byref(gl)))
        return dict(gemm_flops=f.value, gemm_launches=n.value, gemm_ms=ms.value, qr_ms=qms.value,
                    qr_launches=qn.value, qr_gemm_flops=qf.value, masked_launches=mn.value,
                    masked_ms=mms.value, gemm_bytes=gb.value, graph_launches=gl.value)

    def set_timing(self, on: bool):
        self._check(lib().tn_set_timing(self.h, 1 if on else 0))

    def set_autotune(self, on: bool, cache_path: str | None = None):
        """Times the GETT tile configurations on each new contraction shape and
        keeps the fastest (see tn_set_autotune)."""
        self._check(lib().tn_set_autotune(self.h, 1 if on else 0,
                                          None if cache_path is None else cache_path.encode()))

    def plan_report(self, top: int = 30) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(lib().tn_plan_report(self.h, top, buf, len(buf)))
        return buf.value.decode()

    # ---------------------------------------------------------------- test hooks
    def test_sample_config(self, wave: int = 0, rows_limit: int = 0, log_cond=None, graphs: bool = True):
        """Later samples run in waves of `wave` (0 = automatic), stop after
        `rows_limit` rows (0 = all), write log P(x_q | earlier) into log_cond
        (device float64 [n][N]) if given, and replay full waves from a captured
        graph unless graphs is False (see tn_test_sample_config).  The tensor
        must stay alive while the setting is in force."""
        ptr = ctypes.c_void_p(log_cond.data_ptr()) if log_cond is not None else None
        self._check(lib().tn_test_sample_config(self.h, int(wave), int(rows_limit), ptr, 1 if graphs else 0))

    def test_contract(self, prec: str, ia: str, A, ib: str, B, ic: str, C, conjA=False, conjB=False,
                      accumulate=False, cfg: int = -1, ksplit: int = 0, mask=None, mask_letter: str = "z"):
        """C[ic] (+)= A[ia] B[ib] through the contraction engine; with `mask`
        (device int32 over letter mask_letter) the tiles of masked-out items
        are skipped (see tn_test_set_mask)."""
        if mask is not None:
            self._check(lib().tn_test_set_mask(self.h, ctypes.c_void_p(mask.data_ptr()), mask_letter.encode()))
        try:
            self._test_contract(prec, ia, A, ib, B, ic, C, conjA, conjB, accumulate, cfg, ksplit)
        finally:
            if mask is not None:
                lib().tn_test_set_mask(self.h, None, b"z")

    def _test_contract(self, prec, ia, A, ib, B, ic, C, conjA, conjB, accumulate, cfg, ksplit):
        self._check(lib().tn_test_contract(self.h, PREC[prec], ia.encode(), ctypes.c_void_p(A.data_ptr()),
                                           _i32(A.shape), int(conjA), ib.encode(), ctypes.c_void_p(B.data_ptr()),
                                           _i32(B.shape), int(conjB), ic.encode(), ctypes.c_void_p(C.data_ptr()),
                                           _i32(C.shape), int(accumulate), int(cfg), int(ksplit)))

    def test_svd(self, R, cutoff: float, chi_min: int = 1, esz: int = 16):
        """The sampler's SVD truncation on complex128 matrices R [batch][n][n]:
        returns (U, SV, k) with R ~ U @ SV (see tn_test_svd)."""
        import torch
        R = R.to(torch.complex128).contiguous()
        n = R.shape[-1]
        batch = R.shape[0]
        dt = torch.complex128 if esz == 16 else torch.complex64
        U = torch.empty((batch, n, n), dtype=dt, device=R.device)
        SV = torch.empty((batch, n, n), dtype=dt, device=R.device)
        k = torch.empty((batch,), dtype=torch.int32, device=R.device)
        self._check(lib().tn_test_svd(self.h, n, batch, ctypes.c_void_p(R.data_ptr()), float(cutoff), int(chi_min),
                                      ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(SV.data_ptr()), esz,
                                      ctypes.c_void_p(k.data_ptr())))
        return U, SV, k

    def test_qr(self, A, Q, R, method: str | None = None):
        """method "householder" or "cholesky" (default: Householder when R is
        given, CholeskyQR3 otherwise); "cholesky_lq": A and Q are n x m (wide),
        the rows of Q an orthonormal basis of the rows of A, read and written
        through conjugate-transposed strides as in the fit's LQ moves."""
        m, n = A.shape[-2], A.shape[-1]
        if method == "cholesky_lq":
            m, n = n, m
        batch = int(np.prod(A.shape[:-2])) if A.dim() > 2 else 1
        esz = 16 if A.element_size() == 16 else 8
        if method is None:
            method = "householder" if R is not None else "cholesky"
        self._check(lib().tn_test_qr(self.h, m, n, batch, esz, ctypes.c_void_p(A.data_ptr()),
                                     ctypes.c_void_p(Q.data_ptr()),
                                     ctypes.c_void_p(R.data_ptr()) if R is not None else None,
                                     {"householder": 0, "cholesky": 1, "cholesky_lq": 2}[method]))
