"""Python binding of librsdock: argument marshalling only; all work runs in the HIP library.

Arrays may be numpy arrays (host pointers: the call is synchronous and outputs come
back as numpy arrays) or torch CUDA tensors (device pointers: work is enqueued on
the context's stream, outputs are torch CUDA tensors).  Names follow the C ABI in
include/rsdock.h: build_rs_tensor (Algorithm TEP) and score_poses (Algorithm PLIE
with the short-range term and the van der Waals flag).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import FLAG_ACCEPT, FLAG_IN_DOMAIN, FLAG_INVALID, RSD_DEVICE_PTRS, SincParams  # noqa: F401


class RsdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librsdock error {code}: {msg}")
        self.code = code


def _check(status: int) -> None:
    if status != 0:
        raise RsdError(status, _lib.lib().rsd_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _arr(x, dtype=np.float64):
    """(pointer, keepalive, is_device) for a numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        want = {np.float64: torch.float64, np.uint8: torch.uint8, np.int32: torch.int32}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"expected a contiguous torch.{want} tensor")
        return C.c_void_p(x.data_ptr()), x, bool(x.is_cuda)
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(C.c_void_p), a, False


@dataclass
class Sinc:
    """Quadrature (eq. 2.2), range split (eq. 2.4), short-range cutoff and truncation eps."""
    M: int
    h_M: float
    L_s: float
    K_long: int
    r_cut: float
    eps: float

    def c(self) -> SincParams:
        return SincParams(int(self.M), int(self.K_long), float(self.h_M), float(self.L_s),
                          float(self.r_cut), float(self.eps))

    @classmethod
    def from_config(cls, cfg) -> "Sinc":
        return cls(cfg.M, cfg.h_M, cfg.L_s, cfg.K_long, cfg.r_cut, cfg.eps)


class Context:
    """rsd_context: a device, the stream work is enqueued on, and an HBM budget."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except ImportError:
                stream = None
        h = C.c_void_p()
        _check(_lib.lib().rsd_context_create(int(device), C.c_void_p(stream or 0), int(hbm_budget), C.byref(h)))
        self.handle = h
        self._raw = h          # the library keeps a freed context alive while its tensors live
        self.device = device

    def set_stream(self, stream) -> None:
        _check(_lib.lib().rsd_context_set_stream(self.handle, C.c_void_p(stream or 0)))

    def memory(self):
        used, budget = C.c_size_t(), C.c_size_t()
        _check(_lib.lib().rsd_context_memory(self.handle, C.byref(used), C.byref(budget)))
        return used.value, budget.value

    def set_option(self, name: str, value: int) -> None:
        _check(_lib.lib().rsd_context_set_option(self.handle, name.encode(), int(value)))

    def autotune(self, tensor: "Tensor", lig_charges, lig_positions, quats, trans, vdw_min: float,
                 grads: bool = False) -> dict:
        """rsd_autotune on a sample of a workload (device tensors); returns the report as a dict."""
        args = [_arr(x) for x in (lig_charges, lig_positions, quats, trans)]
        if not all(a[2] for a in args):
            raise TypeError("autotune takes device tensors")
        rep = _lib.TuneReport()
        _check(_lib.lib().rsd_autotune(self.handle, tensor.handle, args[0][0], args[1][0], int(args[0][1].shape[0]),
                                       args[2][0], args[3][0], int(args[2][1].shape[0]), float(vdw_min),
                                       int(bool(grads)), C.byref(rep)))
        return {k: getattr(rep, k) for k, _ in _lib.TuneReport._fields_}

    def autotune_cells(self, tensor: "Tensor", lig_charges, lig_positions, quats, trans, vdw_min: float,
                       grads: bool = False) -> dict:
        """rsd_autotune_cells: the cell edge r_cut/div (div 3..6) of the tensor's cell list that
        scores a sample fastest; the tensor keeps it.  Returns dict(div, ms={div: ms})."""
        args = [_arr(x) for x in (lig_charges, lig_positions, quats, trans)]
        if not all(a[2] for a in args):
            raise TypeError("autotune_cells takes device tensors")
        best = C.c_int32()
        ms = (C.c_double * 4)()
        _check(_lib.lib().rsd_autotune_cells(self.handle, tensor.handle, args[0][0], args[1][0],
                                             int(args[0][1].shape[0]), args[2][0], args[3][0],
                                             int(args[2][1].shape[0]), float(vdw_min), int(bool(grads)),
                                             C.byref(best), ms))
        return dict(div=best.value, ms={3 + i: ms[i] for i in range(4)})

    def set_timing(self, enable: bool) -> None:
        _check(_lib.lib().rsd_context_set_timing(self.handle, int(bool(enable))))

    def kernel_time(self, name: str):
        n, ms = C.c_int64(), C.c_double()
        _check(_lib.lib().rsd_kernel_time(self.handle, name.encode(), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def close(self) -> None:
        if getattr(self, "handle", None):
            _lib.lib().rsd_context_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Tensor:
    """rsd_tensor: a resident RS tensor (canonical factors + protein cell list)."""

    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx = ctx
        self.handle = handle

    def query(self):
        n, R, ranks, nbytes = C.c_int32(), C.c_int64(), (C.c_int32 * 3)(), C.c_size_t()
        _check(_lib.lib().rsd_tensor_query(self.handle, C.byref(n), C.byref(R), ranks, C.byref(nbytes)))
        return dict(n=n.value, R=R.value, ranks=tuple(ranks), bytes=nbytes.value)

    def export(self):
        info = self.query()
        F = [np.empty((info["n"], info["R"])) for _ in range(3)]
        _check(_lib.lib().rsd_tensor_export(self.handle, *[f.ctypes.data_as(C.c_void_p) for f in F]))
        return F

    def save(self, path: str) -> None:
        _check(_lib.lib().rsd_tensor_save(self.handle, str(path).encode()))

    def grid(self):
        """rsd_tensor_grid: per-mode origins X0, row counts and the mesh h."""
        X0, rows, h = (C.c_double * 3)(), (C.c_int32 * 3)(), C.c_double()
        _check(_lib.lib().rsd_tensor_grid(self.handle, X0, rows, C.byref(h)))
        return dict(X0=tuple(X0), rows=tuple(rows), h=h.value)

    def restrict(self, lo, hi, eps: float, ctx: "Context" = None) -> "Tensor":
        """rsd_tensor_restrict: this tensor on the sub-box [lo, hi], rank-reduced at eps (Sec. 3.3, scheme (C))."""
        ctx = ctx or self.ctx
        lo3 = (C.c_double * 3)(*[float(x) for x in lo])
        hi3 = (C.c_double * 3)(*[float(x) for x in hi])
        out = C.c_void_p()
        _check(_lib.lib().rsd_tensor_restrict(ctx.handle, self.handle, lo3, hi3, float(eps), C.byref(out)))
        return Tensor(ctx, out)

    def self_energy(self, ctx: "Context" = None):
        """rsd_self_energy: (E_long, E_short) of the molecule itself (Prop. 3.2)."""
        ctx = ctx or self.ctx
        el, es = C.c_double(), C.c_double()
        _check(_lib.lib().rsd_self_energy(ctx.handle, self.handle, C.byref(el), C.byref(es)))
        return el.value, es.value

    def layout(self):
        """rsd_tensor_layout: rank chunks and those whose mode-3 rows come from U_3."""
        nchunk, shared = C.c_int32(), C.c_int32()
        _check(_lib.lib().rsd_tensor_layout(self.handle, C.byref(nchunk), C.byref(shared)))
        return dict(nchunk=nchunk.value, shared_mode3=shared.value)

    def free(self) -> None:
        if getattr(self, "handle", None):
            _lib.lib().rsd_tensor_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _protein_args(charges, positions):
    zp, zk, zdev = _arr(charges)
    xp, xk, xdev = _arr(positions)
    if zdev != xdev:
        raise TypeError("charges and positions must both be host or both be device arrays")
    N = int(zk.shape[0]) if hasattr(zk, "shape") else len(zk)
    return zp, xp, N, (zk, xk), RSD_DEVICE_PTRS if zdev else 0


def build_rs_tensor(ctx: Context, charges, positions, n: int, b: float, sinc: Sinc) -> Tensor:
    """rsd_build_rs_tensor: Algorithm TEP on the device."""
    zp, xp, N, keep, flags = _protein_args(charges, positions)
    out = C.c_void_p()
    sp = sinc.c()
    _check(_lib.lib().rsd_build_rs_tensor(ctx.handle, zp, xp, N, int(n), float(b), C.byref(sp), flags,
                                          C.byref(out)))
    return Tensor(ctx, out)


def pose_order(ctx: Context, tensor: Tensor, quats, trans):
    """rsd_pose_order: (perm, quats in that order, trans in that order, whether scoring these
    poses on this context would sort them itself); device tensors in and out."""
    import torch
    qp, qk, qdev = _arr(quats)
    tp, tk, tdev = _arr(trans)
    if not (qdev and tdev):
        raise TypeError("quats and trans must be device tensors")
    P = int(tk.shape[0])
    perm = torch.empty(P, dtype=torch.int32, device=tk.device)
    q_out = torch.empty_like(qk)
    t_out = torch.empty_like(tk)
    flag = C.c_int32()
    _check(_lib.lib().rsd_pose_order(ctx.handle, tensor.handle, qp, tp, P, C.c_void_p(perm.data_ptr()),
                                     C.c_void_p(q_out.data_ptr()), C.c_void_p(t_out.data_ptr()), C.byref(flag)))
    return perm, q_out, t_out, bool(flag.value)


def tensor_import(ctx: Context, F, n: int, b: float, sinc: Sinc, charges, positions) -> Tensor:
    """rsd_tensor_import: resident tensor from given n x R factors (host arrays)."""
    Fs = [np.ascontiguousarray(f, dtype=np.float64) for f in F]
    R = int(Fs[0].shape[1]) if Fs[0].ndim == 2 else 0
    zp, xp, N, keep, flags = _protein_args(charges, positions)
    if flags:
        raise TypeError("tensor_import from Python takes host arrays")
    out = C.c_void_p()
    sp = sinc.c()
    _check(_lib.lib().rsd_tensor_import(ctx.handle, *[f.ctypes.data_as(C.c_void_p) for f in Fs], R, int(n),
                                        float(b), C.byref(sp), zp, xp, N, 0, C.byref(out)))
    return Tensor(ctx, out)


def tensor_combine(ctx: Context, tensors, eps: float) -> Tensor:
    """rsd_tensor_combine: the potential of a complex of molecules (eq. 5.1), the sum of the
    tensors' canonical terms rank-reduced at eps (add-and-compress); atoms are the union."""
    tensors = list(tensors)
    arr = (C.c_void_p * len(tensors))(*[t.handle for t in tensors])
    out = C.c_void_p()
    _check(_lib.lib().rsd_tensor_combine(ctx.handle, arr, len(tensors), float(eps), C.byref(out)))
    return Tensor(ctx, out)


def tensor_load(ctx: Context, path: str) -> Tensor:
    out = C.c_void_p()
    _check(_lib.lib().rsd_tensor_load(ctx.handle, str(path).encode(), C.byref(out)))
    return Tensor(ctx, out)


def score_poses(ctx: Context, tensor: Tensor, lig_charges, lig_positions, quats, trans, vdw_min: float,
                grads: bool = False, energies_long: bool = False, out: dict | None = None) -> dict:
    """rsd_score_poses.  Returns dict(E, flags, counts[, E_long][, grads])."""
    zp, zk, zdev = _arr(lig_charges)
    lp, lk, ldev = _arr(lig_positions)
    qp, qk, qdev = _arr(quats)
    tp, tk, tdev = _arr(trans)
    if not (zdev == ldev == qdev == tdev):
        raise TypeError("all inputs must be host arrays or all device tensors")
    L = int(zk.shape[0])
    P = int(qk.shape[0])
    if out is None:
        if qdev:
            import torch
            dev = qk.device
            out = dict(E=torch.empty(P, dtype=torch.float64, device=dev),
                       flags=torch.empty(P, dtype=torch.uint8, device=dev),
                       counts=torch.empty(P, dtype=torch.int32, device=dev))
            if energies_long:
                out["E_long"] = torch.empty(P, dtype=torch.float64, device=dev)
            if grads:
                out["grads"] = torch.empty((P, 6), dtype=torch.float64, device=dev)
        else:
            out = dict(E=np.empty(P), flags=np.empty(P, dtype=np.uint8), counts=np.empty(P, dtype=np.int32))
            if energies_long:
                out["E_long"] = np.empty(P)
            if grads:
                out["grads"] = np.empty((P, 6))
    ep = _arr(out["E"])[0]
    fp = _arr(out["flags"], np.uint8)[0]
    cp = _arr(out["counts"], np.int32)[0]
    elp = _arr(out["E_long"])[0] if "E_long" in out else None
    gp = _arr(out["grads"])[0] if "grads" in out else None
    _check(_lib.lib().rsd_score_poses(ctx.handle, tensor.handle, zp, lp, L, qp, tp, P, float(vdw_min),
                                      RSD_DEVICE_PTRS if qdev else 0, ep, elp, fp, cp, gp))
    return out


def probe_gather(ctx: Context, n: int = 2048, iters: int = 256) -> dict:
    """rsd_probe_gather: the long-range kernel's gather pattern alone; bytes, ms and GB/s."""
    ms, nbytes = C.c_double(), C.c_double()
    _check(_lib.lib().rsd_probe_gather(ctx.handle, int(n), int(iters), C.byref(ms), C.byref(nbytes)))
    return dict(ms=ms.value, bytes=nbytes.value, gbs=nbytes.value / (ms.value * 1e-3) / 1e9)


def score_poses_noalloc(ctx: Context, tensor: Tensor, lig_charges, lig_positions, quats, trans, vdw_min: float,
                        out: dict) -> dict:
    """rsd_score_poses_noalloc: rsd_score_poses on device tensors with the library's static
    scratch; `out` holds the caller's output tensors (E, flags, counts[, E_long][, grads])."""
    args = [_arr(x) for x in (lig_charges, lig_positions, quats, trans)]
    if not all(a[2] for a in args):
        raise TypeError("score_poses_noalloc takes device tensors")
    ep = _arr(out["E"])[0]
    fp = _arr(out["flags"], np.uint8)[0]
    cp = _arr(out["counts"], np.int32)[0]
    elp = _arr(out["E_long"])[0] if "E_long" in out else None
    gp = _arr(out["grads"])[0] if "grads" in out else None
    _check(_lib.lib().rsd_score_poses_noalloc(ctx.handle, tensor.handle, args[0][0], args[1][0],
                                              int(args[0][1].shape[0]), args[2][0], args[3][0],
                                              int(args[2][1].shape[0]), float(vdw_min), RSD_DEVICE_PTRS, ep, elp,
                                              fp, cp, gp))
    return out


class Batch:
    """rsd_batch: many requests (device tensors, energies only) scored by one set of launches.

    `requests` is a list of dicts with keys tensor, lig_charges, lig_positions, quats, trans,
    vdw_min and optionally out (dict of E, flags, counts[, E_long] device tensors; allocated
    when absent).  run() only enqueues work, so it can be captured in a HIP graph.
    """

    def __init__(self, ctx: Context, requests: list):
        import torch
        self.ctx = ctx
        self.requests = []
        arr = (_lib.Request * len(requests))()
        for i, r in enumerate(requests):
            q, t = r["quats"], r["trans"]
            P = int(q.shape[0])
            out = r.get("out")
            if out is None:
                dev = q.device
                out = dict(E=torch.empty(P, dtype=torch.float64, device=dev),
                           flags=torch.empty(P, dtype=torch.uint8, device=dev),
                           counts=torch.empty(P, dtype=torch.int32, device=dev))
            keep = dict(r, out=out)
            self.requests.append(keep)
            for x in (r["lig_charges"], r["lig_positions"], q, t, out["E"]):
                if not (_is_torch(x) and x.is_cuda and x.is_contiguous() and x.dtype == torch.float64):
                    raise TypeError("batch arrays must be contiguous float64 device tensors")
            arr[i] = _lib.Request(r["tensor"].handle.value, r["lig_charges"].data_ptr(), r["lig_positions"].data_ptr(),
                                  int(r["lig_charges"].shape[0]), q.data_ptr(), t.data_ptr(), P,
                                  float(r["vdw_min"]), out["E"].data_ptr(),
                                  out["E_long"].data_ptr() if "E_long" in out else None,
                                  out["flags"].data_ptr(), out["counts"].data_ptr())
        h = C.c_void_p()
        _check(_lib.lib().rsd_batch_create(ctx.handle, arr, len(requests), C.byref(h)))
        self.handle = h

    def run(self) -> None:
        _check(_lib.lib().rsd_batch_run(self.handle))

    def outputs(self) -> list:
        return [r["out"] for r in self.requests]

    def free(self) -> None:
        if getattr(self, "handle", None):
            _lib.lib().rsd_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
