"""ctypes binding of libatm3.so (argument marshalling only).

Every step of the computation runs in the HIP kernels of libatm3.so; this
module only passes torch device pointers, sizes and the current HIP stream
across the C ABI declared in include/atm3.h, and turns status codes into
exceptions.  If the library is missing it raises: there is no other path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libatm3.so")

ATM3_OK = 0
ATM3_EINVAL = -1
ATM3_EDEVICE = -2
ATM3_ENOMEM = -3
ATM3_ERANGE = -4
ATM3_EOVERFLOW = -5

TRUNCATIONS = {"pair": 0, "product": 1}
VARIANTS = {"3c08": 0, "3c18": 1, "3c01": 2}
TERM_LJ = 1
TERM_ATM = 2

EXPORTS = (
    "atm3_create", "atm3_destroy", "atm3_set_stream", "atm3_last_error", "atm3_version",
    "atm3_bin_cells", "atm3_compute_forces", "atm3_compute_forces_async",
    "atm3_profile_enable", "atm3_profile_read",
    "atm3_mlp_create", "atm3_mlp_destroy", "atm3_mlp_set_params", "atm3_mlp_get_params",
    "atm3_mlp_set_stats", "atm3_mlp_get_stats", "atm3_mlp_fit_stats", "atm3_surrogate_forces",
    "atm3_mlp_grad", "atm3_mlp_adam", "atm3_mlp_train_step", "atm3_surrogate_pairs",
    "atm3_md_kick_drift", "atm3_md_kick", "atm3_md_kinetic", "atm3_md_rescale", "atm3_md_slab_lrc",
    "atm3_md_nvt_graph", "atm3_virial_diag", "atm3_compute_forces_noalloc",
)
NOALLOC_MAX_N = 65536
NOALLOC_MAX_CELLS = 65536
MLP_NPARAM = 43650
MLP_NDESC = 64
PHASES = {"binning": 0, "block": 1, "big": 2, "reduce": 3}


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("sigma", ctypes.c_double), ("nu", ctypes.c_double),
                ("rc", ctypes.c_double), ("truncation", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("terms", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("e_lj", ctypes.c_double), ("e_atm", ctypes.c_double), ("w_lj", ctypes.c_double),
                ("w_atm", ctypes.c_double), ("n_pairs", ctypes.c_int64), ("n_triplets", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("ncell", ctypes.c_int32 * 3), ("status", ctypes.c_int32)]

    def as_dict(self):
        return {"e_lj": self.e_lj, "e_atm": self.e_atm, "w_lj": self.w_lj, "w_atm": self.w_atm,
                "n_pairs": int(self.n_pairs), "n_triplets": int(self.n_triplets),
                "n_candidates": int(self.n_candidates), "ncell": tuple(self.ncell),
                "status": int(self.status)}


class Atm3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"atm3 error {code}: {msg}")
        self.code = code


_lib = None
_lock = threading.Lock()


def load():
    """Load libatm3.so (raises ImportError if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_2510_21230_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        dptr = ctypes.POINTER(ctypes.c_double)
        iptr = ctypes.POINTER(ctypes.c_int32)
        lib.atm3_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        lib.atm3_create.restype = ctypes.c_int
        lib.atm3_destroy.argtypes = [vp]
        lib.atm3_destroy.restype = None
        lib.atm3_set_stream.argtypes = [vp, vp]
        lib.atm3_set_stream.restype = ctypes.c_int
        lib.atm3_last_error.argtypes = [vp]
        lib.atm3_last_error.restype = ctypes.c_char_p
        lib.atm3_version.argtypes = []
        lib.atm3_version.restype = ctypes.c_char_p
        lib.atm3_bin_cells.argtypes = [vp, vp, i64, dptr, ctypes.c_double, vp, vp, vp, iptr]
        lib.atm3_bin_cells.restype = ctypes.c_int
        lib.atm3_compute_forces.argtypes = [vp, vp, i64, dptr, ctypes.POINTER(Params), vp, ctypes.POINTER(Result)]
        lib.atm3_compute_forces.restype = ctypes.c_int
        lib.atm3_compute_forces_async.argtypes = [vp, vp, i64, dptr, ctypes.POINTER(Params), vp, vp]
        lib.atm3_compute_forces_async.restype = ctypes.c_int
        lib.atm3_compute_forces_noalloc.argtypes = [vp, vp, i64, dptr, ctypes.POINTER(Params), vp, vp]
        lib.atm3_compute_forces_noalloc.restype = ctypes.c_int
        lib.atm3_profile_enable.argtypes = [vp, ctypes.c_int]
        lib.atm3_profile_enable.restype = ctypes.c_int
        lib.atm3_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64)]
        lib.atm3_profile_read.restype = ctypes.c_int
        u64 = ctypes.c_uint64
        fptr = ctypes.POINTER(ctypes.c_float)
        lib.atm3_mlp_create.argtypes = [vp, u64, ctypes.POINTER(vp)]
        lib.atm3_mlp_create.restype = ctypes.c_int
        lib.atm3_mlp_destroy.argtypes = [vp]
        lib.atm3_mlp_destroy.restype = None
        for name in ("atm3_mlp_set_params", "atm3_mlp_get_params"):
            getattr(lib, name).argtypes = [vp, vp, fptr, i64]
            getattr(lib, name).restype = ctypes.c_int
        for name in ("atm3_mlp_set_stats", "atm3_mlp_get_stats"):
            getattr(lib, name).argtypes = [vp, vp, fptr, fptr]
            getattr(lib, name).restype = ctypes.c_int
        lib.atm3_mlp_fit_stats.argtypes = [vp, vp, vp, i64, dptr, ctypes.c_double]
        lib.atm3_mlp_fit_stats.restype = ctypes.c_int
        lib.atm3_surrogate_forces.argtypes = [vp, vp, vp, i64, dptr, ctypes.POINTER(Params), ctypes.c_float, vp, vp,
                                              ctypes.POINTER(Result), ctypes.POINTER(i64)]
        lib.atm3_surrogate_forces.restype = ctypes.c_int
        lib.atm3_mlp_grad.argtypes = [vp, vp, vp, i64, dptr, ctypes.c_double, vp, ctypes.c_float, vp,
                                      ctypes.POINTER(ctypes.c_double)]
        lib.atm3_mlp_grad.restype = ctypes.c_int
        lib.atm3_mlp_adam.argtypes = [vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        lib.atm3_mlp_adam.restype = ctypes.c_int
        lib.atm3_mlp_train_step.argtypes = [vp, vp, vp, i64, dptr, ctypes.c_double, vp, ctypes.c_float,
                                            ctypes.c_float, ctypes.POINTER(ctypes.c_double)]
        lib.atm3_mlp_train_step.restype = ctypes.c_int
        lib.atm3_surrogate_pairs.argtypes = [vp, vp, vp, i64, dptr, ctypes.c_double, i64, vp, vp, vp, vp, vp,
                                             ctypes.POINTER(i64)]
        lib.atm3_surrogate_pairs.restype = ctypes.c_int
        lib.atm3_md_kick_drift.argtypes = [vp, vp, vp, vp, i64, ctypes.c_double]
        lib.atm3_md_kick_drift.restype = ctypes.c_int
        lib.atm3_md_kick.argtypes = [vp, vp, vp, i64, ctypes.c_double]
        lib.atm3_md_kick.restype = ctypes.c_int
        lib.atm3_md_kinetic.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_double)]
        lib.atm3_md_kinetic.restype = ctypes.c_int
        lib.atm3_md_rescale.argtypes = [vp, vp, i64, ctypes.c_double, i64]
        lib.atm3_md_rescale.restype = ctypes.c_int
        lib.atm3_md_slab_lrc.argtypes = [vp, vp, i64, dptr, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, vp, vp]
        lib.atm3_md_slab_lrc.restype = ctypes.c_int
        lib.atm3_md_nvt_graph.argtypes = [vp, vp, vp, i64, dptr, ctypes.POINTER(Params), i64, ctypes.c_double,
                                          ctypes.c_double, i64, i64, vp, vp, i64, ctypes.c_int32, vp]
        lib.atm3_md_nvt_graph.restype = ctypes.c_int
        lib.atm3_virial_diag.argtypes = [vp, vp, i64, dptr, ctypes.POINTER(Params), dptr]
        lib.atm3_virial_diag.restype = ctypes.c_int
        _lib = lib
        return lib


def _box(box):
    b = [float(v) for v in (box if hasattr(box, "__len__") else (box, box, box))]
    if len(b) != 3:
        raise ValueError("box must have 3 lengths")
    return (ctypes.c_double * 3)(*b)


def make_params(rc=2.5, nu=0.073, eps=1.0, sigma=1.0, truncation="pair", variant="3c08",
                terms=TERM_LJ | TERM_ATM, check_finite=False) -> Params:
    return Params(float(eps), float(sigma), float(nu), float(rc), TRUNCATIONS[truncation],
                  VARIANTS[variant], int(terms), 2 if check_finite else 0)


class Context:
    """One libatm3 context (device scratch owner) on a torch CUDA/HIP device."""

    def __init__(self, device=None):
        import torch
        self.lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        rc = self.lib.atm3_create(ctypes.byref(h), self.device.index or 0)
        if rc != ATM3_OK:
            raise Atm3Error(rc, f"atm3_create failed for {self.device}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.atm3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != ATM3_OK:
            msg = self.lib.atm3_last_error(self.h).decode(errors="replace")
            if rc == ATM3_EINVAL:
                raise ValueError(msg)
            raise Atm3Error(rc, msg)

    def _stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.atm3_set_stream(self.h, ctypes.c_void_p(s)))

    def _pos(self, pos):
        import torch
        if not (pos.is_cuda and pos.dtype == torch.float64 and pos.dim() == 2 and pos.shape[1] == 3):
            raise ValueError("pos must be a (N,3) float64 tensor on the GPU")
        if pos.device != self.device:
            raise ValueError(f"pos is on {pos.device}, context on {self.device}")
        return pos.contiguous()

    def bin_cells(self, pos, box, rc):
        """Cell of each molecule, cell_start, perm (sorted slot -> input index), ncell."""
        import torch
        pos = self._pos(pos)
        b = _box(box)
        nc = (ctypes.c_int32 * 3)()
        self._check(self.lib.atm3_bin_cells(self.h, None, 0, b, float(rc), None, None, None, nc))
        ncells = nc[0] * nc[1] * nc[2]
        n = pos.shape[0]
        cell_of = torch.empty(n, dtype=torch.int32, device=self.device)
        start = torch.empty(ncells + 1, dtype=torch.int32, device=self.device)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        self._stream()
        self._check(self.lib.atm3_bin_cells(self.h, ctypes.c_void_p(pos.data_ptr()), n, b, float(rc),
                                            ctypes.c_void_p(cell_of.data_ptr()),
                                            ctypes.c_void_p(start.data_ptr()),
                                            ctypes.c_void_p(perm.data_ptr()), nc))
        return cell_of, start, perm, tuple(nc)

    def compute_forces(self, pos, box, forces=None, **kw):
        """Forces (N,3) float32 in input order and the result dict; blocks."""
        import torch
        pos = self._pos(pos)
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        p = make_params(**kw)
        r = Result()
        self._stream()
        self._check(self.lib.atm3_compute_forces(self.h, ctypes.c_void_p(pos.data_ptr()), n, _box(box),
                                                 ctypes.byref(p), ctypes.c_void_p(forces.data_ptr()),
                                                 ctypes.byref(r)))
        return forces, r.as_dict()

    def virial_diag(self, pos, box, **kw):
        """Diagonal of the virial tensor: (w_lj[3], w_atm[3]) as float64
        arrays (xx, yy, zz); blocks."""
        import numpy as np
        pos = self._pos(pos)
        p = make_params(**kw)
        w = (ctypes.c_double * 6)()
        self._stream()
        self._check(self.lib.atm3_virial_diag(self.h, ctypes.c_void_p(pos.data_ptr()), pos.shape[0], _box(box),
                                              ctypes.byref(p), w))
        return np.array(w[:3]), np.array(w[3:])

    def compute_forces_async(self, pos, box, forces, result_dev, params: Params):
        """Enqueue one evaluation on the current stream; result_dev is a device
        tensor of at least sizeof(atm3_result) bytes."""
        n = pos.shape[0]
        self._stream()
        self._check(self.lib.atm3_compute_forces_async(
            self.h, ctypes.c_void_p(pos.data_ptr()), n, _box(box), ctypes.byref(params),
            ctypes.c_void_p(forces.data_ptr()), ctypes.c_void_p(result_dev.data_ptr())))

    def compute_forces_noalloc(self, pos, box, forces, result_dev, params: Params):
        """As compute_forces_async, with every scratch buffer in the library's
        fixed device array (no device allocation; pairwise cutoff, at most
        NOALLOC_MAX_N molecules and NOALLOC_MAX_CELLS cells)."""
        n = pos.shape[0]
        self._stream()
        self._check(self.lib.atm3_compute_forces_noalloc(
            self.h, ctypes.c_void_p(pos.data_ptr()), n, _box(box), ctypes.byref(params),
            ctypes.c_void_p(forces.data_ptr()), ctypes.c_void_p(result_dev.data_ptr())))

    def slab_lrc(self, pos, box, forces, nbins=600, rc=2.5, eps=1.0, sigma=1.0, hist_sum=None):
        """Add the planar long-range correction of the LJ force to the z
        components of `forces` (enqueued); `hist_sum` (int64, nbins) gets this
        configuration's z histogram added."""
        import torch
        pos = self._pos(pos)
        if not (forces.is_cuda and forces.dtype == torch.float32 and forces.is_contiguous()
                and forces.shape == pos.shape):
            raise ValueError("forces must be a contiguous float32 device tensor shaped like pos")
        if hist_sum is not None and not (hist_sum.is_cuda and hist_sum.dtype == torch.int64
                                         and hist_sum.is_contiguous() and hist_sum.numel() == nbins):
            raise ValueError("hist_sum must be a contiguous int64 device tensor of nbins entries")
        self._stream()
        self._check(self.lib.atm3_md_slab_lrc(self.h, ctypes.c_void_p(pos.data_ptr()), pos.shape[0], _box(box),
                                              int(nbins), float(rc), float(eps), float(sigma),
                                              ctypes.c_void_p(forces.data_ptr()),
                                              None if hist_sum is None else ctypes.c_void_p(hist_sum.data_ptr())))

    def profile(self, enable: bool):
        """Start (clearing totals) or stop HIP-event timing of the kernel phases."""
        self._stream()
        self._check(self.lib.atm3_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{phase: (total_ms, launches)} of the event-timed kernel phases."""
        out = {}
        for name, ph in PHASES.items():
            ms = ctypes.c_double()
            k = ctypes.c_int64()
            self._check(self.lib.atm3_profile_read(self.h, ph, ctypes.byref(ms), ctypes.byref(k)))
            out[name] = (ms.value, int(k.value))
        return out


def result_from_bytes(buf: bytes) -> dict:
    """Decode a device result (copied to host bytes) into a dict."""
    r = Result.from_buffer_copy(buf[:ctypes.sizeof(Result)])
    return r.as_dict()


_ctxs = {}


def context(device=None) -> Context:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    key = torch.device("cuda", device).index if isinstance(device, int) else torch.device(device).index
    if key not in _ctxs:
        _ctxs[key] = Context(key)
    return _ctxs[key]


def bin_cells(pos, box, rc=2.5):
    return context(pos.device).bin_cells(pos, box, rc)


def compute_forces(pos, box, rc=2.5, nu=0.073, eps=1.0, sigma=1.0, truncation="pair",
                   variant="3c08", terms=TERM_LJ | TERM_ATM, check_finite=False, forces=None):
    """Linked-cell LJ + ATM forces of a periodic system on the GPU.

    Returns (forces[N,3] float32, result dict with e_lj, e_atm, w_lj, w_atm,
    n_pairs, n_triplets, n_candidates, ncell)."""
    return context(pos.device).compute_forces(pos, box, forces=forces, rc=rc, nu=nu, eps=eps, sigma=sigma,
                                              truncation=truncation, variant=variant, terms=terms,
                                              check_finite=check_finite)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Mlp:
    """The learned pair surrogate (parameters, Adam state, BF16 copies) on one
    device; every computation runs in libatm3's kernels."""

    def __init__(self, seed=0, device=None):
        self.ctx = context(device)
        self.lib = self.ctx.lib
        h = ctypes.c_void_p()
        self.ctx._check(self.lib.atm3_mlp_create(self.ctx.h, ctypes.c_uint64(seed), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.atm3_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_get_params(self.ctx.h, self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                     MLP_NPARAM))
        return out

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_set_params(self.ctx.h, self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                     MLP_NPARAM))

    def get_stats(self):
        import numpy as np
        m = np.zeros(64, dtype=np.float32)
        s = np.zeros(64, dtype=np.float32)
        self.ctx._stream()
        fp = ctypes.POINTER(ctypes.c_float)
        self.ctx._check(self.lib.atm3_mlp_get_stats(self.ctx.h, self.h, m.ctypes.data_as(fp), s.ctypes.data_as(fp)))
        return m, s

    def set_stats(self, mean, inv_sd):
        import numpy as np
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(inv_sd, dtype=np.float32)
        if m.size != 64 or s.size != 64:
            raise ValueError("statistics have 64 entries each")
        self.ctx._stream()
        fp = ctypes.POINTER(ctypes.c_float)
        self.ctx._check(self.lib.atm3_mlp_set_stats(self.ctx.h, self.h, m.ctypes.data_as(fp), s.ctypes.data_as(fp)))

    def fit_stats(self, pos, box, rc=2.5):
        pos = self.ctx._pos(pos)
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_fit_stats(self.ctx.h, self.h, _ptr(pos), pos.shape[0], _box(box), float(rc)))

    def forces(self, pos, box, threshold=float("inf"), rc=2.5, nu=0.073, eps=1.0, sigma=1.0, want_err=False,
               forces=None):
        """LJ + surrogate three-body forces (exact ATM where the error estimate
        exceeds `threshold`); returns (forces, result dict, n_fallback, err)."""
        import torch
        pos = self.ctx._pos(pos)
        n = pos.shape[0]
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
        err = torch.empty(n, dtype=torch.float32, device=pos.device) if want_err else None
        p = make_params(rc=rc, nu=nu, eps=eps, sigma=sigma)
        r = Result()
        nf = ctypes.c_int64()
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_surrogate_forces(self.ctx.h, self.h, _ptr(pos), n, _box(box), ctypes.byref(p),
                                                       float(threshold), _ptr(forces), _ptr(err), ctypes.byref(r),
                                                       ctypes.byref(nf)))
        return forces, r.as_dict(), int(nf.value), err

    def grad(self, pos, box, target, lam=1.0, rc=2.5, with_grad=True):
        """(gradient tensor or None, loss) of the training loss at one configuration."""
        import torch
        pos = self.ctx._pos(pos)
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=pos.device) if with_grad else None
        loss = ctypes.c_double()
        tgt = target.contiguous()
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_grad(self.ctx.h, self.h, _ptr(pos), pos.shape[0], _box(box), float(rc),
                                               _ptr(tgt), float(lam), _ptr(g), ctypes.byref(loss)))
        return g, loss.value

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_adam(self.ctx.h, self.h, _ptr(grad.contiguous()), float(lr), float(beta1),
                                               float(beta2), float(eps)))

    def train_step(self, pos, box, target, lam=1.0, lr=1e-3, rc=2.5):
        pos = self.ctx._pos(pos)
        loss = ctypes.c_double()
        tgt = target.contiguous()
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_mlp_train_step(self.ctx.h, self.h, _ptr(pos), pos.shape[0], _box(box),
                                                     float(rc), _ptr(tgt), float(lam), float(lr),
                                                     ctypes.byref(loss)))
        return loss.value

    def pairs(self, pos, box, rc=2.5, cap=None):
        """Per-pair outputs and per-molecule descriptors / force / error
        estimate of one evaluation, for inspection (input order)."""
        import torch
        pos = self.ctx._pos(pos)
        n = pos.shape[0]
        npairs = ctypes.c_int64()
        self.ctx._stream()
        self.ctx._check(self.lib.atm3_surrogate_pairs(self.ctx.h, self.h, _ptr(pos), n, _box(box), float(rc), 0,
                                                      None, None, None, None, None, ctypes.byref(npairs)))
        P = npairs.value if cap is None else min(cap, npairs.value)
        dev = pos.device
        ij = torch.empty((max(P, 1), 2), dtype=torch.int32, device=dev)
        st = torch.empty((max(P, 1), 2), dtype=torch.float32, device=dev)
        desc = torch.empty((n, 64), dtype=torch.float32, device=dev)
        f3 = torch.empty((n, 3), dtype=torch.float32, device=dev)
        err = torch.empty(n, dtype=torch.float32, device=dev)
        self.ctx._check(self.lib.atm3_surrogate_pairs(self.ctx.h, self.h, _ptr(pos), n, _box(box), float(rc), P,
                                                      _ptr(ij), _ptr(st), _ptr(desc), _ptr(f3), _ptr(err),
                                                      ctypes.byref(npairs)))
        return {"pair_ij": ij[:P], "st": st[:P], "desc": desc, "f3": f3, "err": err, "n_pairs": npairs.value}


def md_run(pos, vel, box, steps, dt=0.002, record_every=1, frames=None, **force_kw):
    """Velocity Verlet (NVE) for `steps` steps, updating the FP64 device
    tensors `pos` and `vel` in place, with forces from atm3_compute_forces.
    Returns the per-recorded-step dicts (step, kinetic, e_lj, e_atm, total);
    if `frames` is a list, copies of (pos, forces) at the recorded steps are
    appended to it."""
    import torch
    ctx = context(pos.device)
    lib = ctx.lib
    if not (vel.is_cuda and vel.dtype == torch.float64 and vel.shape == pos.shape and vel.is_contiguous()):
        raise ValueError("vel must be a contiguous float64 tensor shaped like pos")
    if not pos.is_contiguous():
        raise ValueError("pos must be contiguous")
    n = pos.shape[0]
    f, r = ctx.compute_forces(pos, box, **force_kw)
    out = []

    def record(k, res):
        ke = ctypes.c_double()
        ctx._check(lib.atm3_md_kinetic(ctx.h, _ptr(vel), n, ctypes.byref(ke)))
        out.append({"step": k, "kinetic": ke.value, "e_lj": res["e_lj"], "e_atm": res["e_atm"],
                    "total": ke.value + res["e_lj"] + res["e_atm"]})
        if frames is not None:
            frames.append((pos.clone(), f.clone()))

    record(0, r)
    for k in range(1, steps + 1):
        ctx._stream()
        ctx._check(lib.atm3_md_kick_drift(ctx.h, _ptr(pos), _ptr(vel), _ptr(f), n, float(dt)))
        f, r = ctx.compute_forces(pos, box, forces=f, **force_kw)
        ctx._check(lib.atm3_md_kick(ctx.h, _ptr(vel), _ptr(f), n, float(dt)))
        if k % record_every == 0:
            record(k, r)
    return out


def md_nvt(pos, vel, box, steps, dt, temperature, sample_every=1, lrc_bins=0, profile=None, graph=False,
           **force_kw):
    """Velocity Verlet with isokinetic rescaling to `temperature` after every
    step (3N - 3 degrees of freedom), updating the FP64 device tensors `pos`
    and `vel` in place; force_kw go to make_params.  Nothing synchronises with
    the host inside the loop: each sampled step's result struct is written to
    its own device row.  Returns a float64 array (n_samples, 4) with the
    atm3_result fields e_lj, e_atm, w_lj, w_atm at steps sample_every,
    2 sample_every, ...  With lrc_bins > 0 every force evaluation gets the
    planar long-range correction of the LJ force on that many z bins, and
    `profile` (int64 device tensor of lrc_bins, if given) accumulates the z
    histogram of every step.  With graph=True one step is captured as a HIP
    graph and launched `steps` times (atm3_md_nvt_graph): same trajectory
    and results, without the per-step host launches."""
    import torch
    ctx = context(pos.device)
    lib = ctx.lib
    if not (vel.is_cuda and vel.dtype == torch.float64 and vel.shape == pos.shape and vel.is_contiguous()):
        raise ValueError("vel must be a contiguous float64 tensor shaped like pos")
    if not pos.is_contiguous():
        raise ValueError("pos must be contiguous")
    n = pos.shape[0]
    prm = make_params(**force_kw)
    f = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    stride = 128  # bytes per result row (>= sizeof(atm3_result), aligned)
    ns = steps // sample_every
    lrc = dict(rc=prm.rc, eps=prm.eps, sigma=prm.sigma)
    if profile is not None and not (profile.is_cuda and profile.dtype == torch.int64 and profile.is_contiguous()
                                    and profile.numel() == lrc_bins):
        raise ValueError("profile must be a contiguous int64 device tensor of lrc_bins entries")
    if graph:
        # rows 0..ns-1: sampled steps; row ns: status folded over every step
        rows = torch.zeros((ns + 1) * stride, dtype=torch.uint8, device=pos.device)
        ctx._stream()
        ctx._check(lib.atm3_md_nvt_graph(ctx.h, _ptr(pos), _ptr(vel), n, _box(box), ctypes.byref(prm), int(steps),
                                         float(dt), float(temperature), 3 * n - 3, int(sample_every), _ptr(f),
                                         _ptr(rows), stride, int(lrc_bins),
                                         None if profile is None else _ptr(profile)))
        return _rows_out(rows, stride, [q for q in range(ns)], [ns])
    # one row per step (row k-1 for step k) and row `steps` for the initial
    # forces, so that every evaluation's status is checked, sampled or not
    rows = torch.zeros((steps + 1) * stride, dtype=torch.uint8, device=pos.device)
    ctx.compute_forces_async(pos, box, f, rows[steps * stride:], prm)
    if lrc_bins:
        ctx.slab_lrc(pos, box, f, lrc_bins, **lrc)
    for k in range(1, steps + 1):
        ctx._check(lib.atm3_md_kick_drift(ctx.h, _ptr(pos), _ptr(vel), _ptr(f), n, float(dt)))
        ctx.compute_forces_async(pos, box, f, rows[(k - 1) * stride:], prm)
        if lrc_bins:
            ctx.slab_lrc(pos, box, f, lrc_bins, hist_sum=profile, **lrc)
        ctx._check(lib.atm3_md_kick(ctx.h, _ptr(vel), _ptr(f), n, float(dt)))
        ctx._check(lib.atm3_md_rescale(ctx.h, _ptr(vel), n, float(temperature), 3 * n - 3))
    return _rows_out(rows, stride, [sample_every * (q + 1) - 1 for q in range(ns)], range(steps + 1))


def _rows_out(rows, stride, sampled, checked):
    """(len(sampled), 4) e_lj, e_atm, w_lj, w_atm of the result rows with the
    indices `sampled`; raises if any row of `checked` holds a failed status."""
    import torch
    torch.cuda.synchronize(rows.device)
    return rows_from_bytes(rows.cpu().numpy().tobytes(), stride, sampled, checked)


def rows_from_bytes(host: bytes, stride, sampled, checked):
    """Host part of _rows_out: decode result rows from raw bytes."""
    import numpy as np
    size = ctypes.sizeof(Result)

    def row(q):
        return Result.from_buffer_copy(host[q * stride:q * stride + size])

    for q in checked:
        st = int(row(q).status)
        if st != 0:
            raise Atm3Error(st, f"force evaluation of row {q} returned status {st}")
    out = np.zeros((len(sampled), 4))
    for a, q in enumerate(sampled):
        r = row(q)
        out[a] = (r.e_lj, r.e_atm, r.w_lj, r.w_atm)
    return out
