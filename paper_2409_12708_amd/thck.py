"""ctypes binding of libthck.so (the C ABI in include/thck.h).

Argument marshalling only: every step of H|psi>, the sums, overlaps and the
Lanczos step runs inside libthck's HIP kernels.  PyTorch provides device
memory (a flat float64 tensor per MPS) and the current HIP stream.  There is
no CPU fallback: if the library is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthck.so")

THC_OK, THC_EINVAL, THC_ENOMEM, THC_EDEVICE, THC_ENONFINITE, THC_ENOCONV, THC_ECAPACITY = 0, -1, -2, -3, -4, -5, -6
PREC = {"f64": 0, "f32": 1, "bf16x3": 2}


class ThcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"thck status {status}: {msg}")
        self.status = status


class ThcMps(C.Structure):
    _fields_ = [
        ("n_sites", C.c_int32),
        ("d", C.c_int32),
        ("bonds", C.POINTER(C.c_int32)),
        ("offsets", C.POINTER(C.c_int64)),
        ("data", C.c_void_p),
        ("capacity", C.c_int64),
        ("canonical", C.c_int32),
        ("reserved", C.c_int32),
    ]


class ThcOpts(C.Structure):
    _fields_ = [
        ("D_max", C.c_int32),
        ("D_sum", C.c_int32),
        ("rel_cutoff", C.c_double),
        ("prec", C.c_int32),
        ("batch", C.c_int32),
        ("max_sweeps", C.c_int32),
        ("include_T", C.c_int32),
        ("include_V", C.c_int32),
        ("flags", C.c_uint64),
    ]


NK = 8  # kernel classes of thc_stats (THC_NK)


class ThcStats(C.Structure):
    _fields_ = [
        ("discarded_weight_max", C.c_double),
        ("flops_model", C.c_double),
        ("n_compressions", C.c_int64),
        ("n_launches", C.c_int64),
        ("max_bond", C.c_int32),
        ("jacobi_sweeps_max", C.c_int32),
        ("nonconverged", C.c_int32),
        ("svd_fallbacks", C.c_int32),
        ("kernel_ms", C.c_double * NK),
        ("kernel_flops", C.c_double * NK),
        ("kernel_launches", C.c_int64 * NK),
        ("kernel_bytes", C.c_double * NK),
        ("graph_captures", C.c_int64),
        ("graph_replays", C.c_int64),
    ]
    KERNELS = ("lq", "sytrd", "tri_eig", "ormtr", "gemm", "svd_fallback", "sb2st", "q2")

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("kernel_")}

    def kernels(self):
        """Per kernel class: (summed ms, algorithmic flops, launches, algorithmic bytes);
        filled with THC_FLAG_TIME_KERNELS."""
        return {k: (self.kernel_ms[i], self.kernel_flops[i], self.kernel_launches[i], self.kernel_bytes[i])
                for i, k in enumerate(self.KERNELS)}


FLAG_SVD_JACOBI = 1      # one-sided Jacobi SVD in the truncation step
FLAG_TIME_KERNELS = 2    # per-kernel-class device times / flops in ThcStats.kernels()
FLAG_GRAPHS = 4          # compression batches captured into HIP graphs and replayed
FLAG_SYTRD_ONE_STAGE = 8  # one-stage tridiagonalisation in the SVD step (default: two stages)
FLAG_TWO_STREAMS = 16    # H applied as two halves (split by nu) on two streams, then added

EXPORTS = [
    "thc_default_opts", "thc_mps_capacity", "thc_load_factors", "thc_destroy", "mps_apply_thc_H",
    "mps_sum_compress", "mps_overlap", "krylov_create", "krylov_destroy", "krylov_step",
    "krylov_get_vector", "krylov_get_matrices", "mps_compress", "mps_apply_layer", "thc_last_error",
    "krylov_ritz_vector", "krylov_restart", "thc_energy_gradient", "mps_overlap_noalloc", "krylov_evolve",
    "mps_sum_compress_complex", "mps_overlap_complex",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libthck.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    lib.thc_default_opts.argtypes = [P(ThcOpts), C.c_int32]
    lib.thc_default_opts.restype = None
    lib.thc_mps_capacity.argtypes = [C.c_int32, C.c_int32]
    lib.thc_mps_capacity.restype = C.c_int64
    lib.thc_load_factors.argtypes = [P(vp), C.c_int32, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double),
                                     C.c_uint64, vp]
    lib.thc_destroy.argtypes = [vp]
    lib.mps_apply_thc_H.argtypes = [vp, P(ThcMps), P(ThcMps), P(ThcOpts), P(ThcStats), vp]
    lib.mps_sum_compress.argtypes = [vp, C.c_int32, P(C.c_double), P(P(ThcMps)), P(ThcMps), P(ThcOpts),
                                     P(ThcStats), vp]
    lib.mps_overlap.argtypes = [vp, P(ThcMps), P(ThcMps), P(C.c_double), vp]
    lib.krylov_create.argtypes = [vp, P(ThcMps), C.c_int32, P(ThcOpts), P(vp), vp]
    lib.krylov_destroy.argtypes = [vp]
    lib.krylov_step.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double), P(ThcStats), vp]
    lib.krylov_get_vector.argtypes = [vp, C.c_int32, P(ThcMps), vp]
    lib.krylov_get_matrices.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_int32)]
    lib.mps_compress.argtypes = [vp, P(ThcMps), P(ThcMps), P(ThcOpts), P(ThcStats), vp]
    lib.mps_apply_layer.argtypes = [vp, P(ThcMps), P(C.c_double), C.c_int32, P(ThcMps), P(ThcOpts),
                                    P(ThcStats), vp]
    lib.krylov_ritz_vector.argtypes = [vp, C.c_int32, P(ThcMps), vp]
    lib.krylov_restart.argtypes = [vp, C.c_int32, vp]
    lib.mps_overlap_noalloc.argtypes = [P(ThcMps), P(ThcMps), vp, vp]
    lib.thc_energy_gradient.argtypes = [vp, P(ThcMps), C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double), vp]
    lib.krylov_evolve.argtypes = [C.c_int32, P(vp), P(P(ThcMps)), P(P(ThcMps)), P(ThcOpts), C.c_int32, C.c_double,
                                  C.c_int32, P(P(ThcMps)), P(P(ThcMps)), P(C.c_int32), P(ThcStats), vp]
    lib.mps_sum_compress_complex.argtypes = [vp, C.c_int32, P(C.c_double), P(P(ThcMps)), P(P(ThcMps)), P(ThcMps),
                                             P(ThcMps), P(ThcOpts), P(ThcStats), vp]
    lib.mps_overlap_complex.argtypes = [vp, P(ThcMps), P(ThcMps), P(ThcMps), P(ThcMps), P(C.c_double), vp]
    lib.thc_last_error.argtypes = []
    lib.thc_last_error.restype = C.c_char_p
    for name in ("thc_load_factors", "thc_destroy", "mps_apply_thc_H", "mps_sum_compress", "mps_overlap",
                 "krylov_create", "krylov_destroy", "krylov_step", "krylov_get_vector", "krylov_get_matrices",
                 "mps_compress", "mps_apply_layer", "krylov_ritz_vector", "krylov_restart",
                 "thc_energy_gradient", "mps_overlap_noalloc", "krylov_evolve", "mps_sum_compress_complex",
                 "mps_overlap_complex"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != THC_OK:
        raise ThcError(status, load_library().thc_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a: np.ndarray):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))


def capacity(n_sites: int, D: int) -> int:
    return int(load_library().thc_mps_capacity(n_sites, D))


def make_opts(D: int, **kw) -> ThcOpts:
    o = ThcOpts()
    load_library().thc_default_opts(C.byref(o), int(D))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        setattr(o, k, v)
    return o


class DeviceMPS:
    """An MPS held in one flat float64 device tensor (site j at offsets[j],
    shaped (bonds[j], 2, bonds[j+1]), row-major)."""

    def __init__(self, n_sites: int, capacity_elems: int, device="cuda"):
        self.n = int(n_sites)
        self.buf = torch.zeros(max(1, int(capacity_elems)), dtype=torch.float64, device=device)
        self.bonds = (C.c_int32 * (self.n + 1))(*([1] * (self.n + 1)))
        self.offsets = (C.c_int64 * self.n)()
        for j in range(self.n):
            self.offsets[j] = 2 * j
        # sites 1..n-1 right-canonical (declared by the caller, or set by the
        # library on the MPS it writes)
        self.canonical = False

    @classmethod
    def from_sites(cls, sites, device="cuda", capacity_elems=None, canonical=False):
        n = len(sites)
        sizes = [int(np.prod(a.shape)) for a in sites]
        cap = sum(sizes) if capacity_elems is None else max(capacity_elems, sum(sizes))
        m = cls(n, cap, device)
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in sites])
        m.buf[: flat.size].copy_(torch.from_numpy(flat))
        o = 0
        for j, a in enumerate(sites):
            m.bonds[j] = a.shape[0]
            m.offsets[j] = o
            o += sizes[j]
        m.bonds[n] = sites[-1].shape[2]
        m.canonical = bool(canonical)
        return m

    def bond_list(self):
        return [int(self.bonds[j]) for j in range(self.n + 1)]

    def to_sites(self):
        host = self.buf.detach().cpu().numpy()
        out = []
        for j in range(self.n):
            l, r = int(self.bonds[j]), int(self.bonds[j + 1])
            o = int(self.offsets[j])
            out.append(host[o:o + l * 2 * r].reshape(l, 2, r).copy())
        return out

    def desc(self) -> ThcMps:
        d = ThcMps()
        d.n_sites = self.n
        d.d = 2
        d.bonds = C.cast(self.bonds, C.POINTER(C.c_int32))
        d.offsets = C.cast(self.offsets, C.POINTER(C.c_int64))
        d.data = C.c_void_p(self.buf.data_ptr())
        d.capacity = self.buf.numel()
        d.canonical = int(bool(self.canonical))
        d.reserved = 0
        return d

    def _written(self, d: ThcMps) -> "DeviceMPS":
        self.canonical = bool(d.canonical)
        return self


class Context:
    """THC factors loaded on the device (thc_load_factors)."""

    def __init__(self, t, chi, zeta, device="cuda"):
        self.lib = load_library()
        t = np.ascontiguousarray(t, dtype=np.float64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        zeta = np.ascontiguousarray(zeta, dtype=np.float64)
        self.L, self.N = chi.shape
        self.n = 2 * self.L
        self.device = device
        self._keep = (t, chi, zeta)
        h = C.c_void_p()
        _check(self.lib.thc_load_factors(C.byref(h), self.L, self.N, _dptr(t), _dptr(chi), _dptr(zeta), 0,
                                         _stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.thc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_mps(self, D: int) -> DeviceMPS:
        return DeviceMPS(self.n, capacity(self.n, D), self.device)

    def apply_H(self, psi: DeviceMPS, D: int, stats: ThcStats | None = None, **kw) -> DeviceMPS:
        o = make_opts(D, **kw)
        out = self.new_mps(D)
        pd, od = psi.desc(), out.desc()
        _check(self.lib.mps_apply_thc_H(self.h, C.byref(pd), C.byref(od), C.byref(o),
                                        C.byref(stats) if stats is not None else None, _stream()))
        return out._written(od)

    def sum_compress(self, coeffs, terms, D: int, stats: ThcStats | None = None, **kw) -> DeviceMPS:
        o = make_opts(D, **kw)
        k = len(terms)
        descs = [t.desc() for t in terms]
        arr = (C.POINTER(ThcMps) * k)(*[C.pointer(d) for d in descs])
        co = (C.c_double * k)(*[float(c) for c in coeffs])
        out = self.new_mps(D)
        od = out.desc()
        _check(self.lib.mps_sum_compress(self.h, k, co, arr, C.byref(od), C.byref(o),
                                         C.byref(stats) if stats is not None else None, _stream()))
        return out._written(od)

    def compress(self, psi: DeviceMPS, D: int, stats: ThcStats | None = None, **kw) -> DeviceMPS:
        o = make_opts(D, **kw)
        out = self.new_mps(D)
        pd, od = psi.desc(), out.desc()
        _check(self.lib.mps_compress(self.h, C.byref(pd), C.byref(od), C.byref(o),
                                     C.byref(stats) if stats is not None else None, _stream()))
        return out._written(od)

    def apply_layer(self, psi: DeviceMPS, y, dag: bool, D: int, stats: ThcStats | None = None, **kw) -> DeviceMPS:
        o = make_opts(D, **kw)
        out = self.new_mps(D)
        y = np.ascontiguousarray(y, dtype=np.float64)
        pd, od = psi.desc(), out.desc()
        _check(self.lib.mps_apply_layer(self.h, C.byref(pd), _dptr(y), int(bool(dag)), C.byref(od), C.byref(o),
                                        C.byref(stats) if stats is not None else None, _stream()))
        return out._written(od)

    def energy_gradient(self, psi: DeviceMPS, prec="f64"):
        """(E, dE/dchi (L x N), dE/dzeta (N x N)) of E = <psi|H|psi> for the
        loaded factors (thc_energy_gradient)."""
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        e = C.c_double()
        dchi = np.zeros((self.L, self.N))
        dzeta = np.zeros((self.N, self.N))
        pd = psi.desc()
        _check(self.lib.thc_energy_gradient(self.h, C.byref(pd), p, C.byref(e), _dptr(dchi), _dptr(dzeta),
                                            _stream()))
        return float(e.value), dchi, dzeta

    def sum_compress_complex(self, coeffs, terms, D: int, stats: ThcStats | None = None, **kw):
        """Compressed sum_i c_i |t_i> for complex c_i and complex states given as
        (re, im) pairs of DeviceMPS (None = zero part); returns an (re, im) pair."""
        o = make_opts(D, **kw)
        k = len(terms)
        keep = []

        def ptr(m):
            if m is None:
                return None
            d = m.desc()
            keep.append(d)
            return C.pointer(d)

        re_arr = (C.POINTER(ThcMps) * k)(*[ptr(t[0]) for t in terms])
        im_arr = (C.POINTER(ThcMps) * k)(*[ptr(t[1]) for t in terms])
        co = (C.c_double * (2 * k))(*[v for c in coeffs for v in (complex(c).real, complex(c).imag)])
        out_re, out_im = self.new_mps(D), self.new_mps(D)
        dr, di = out_re.desc(), out_im.desc()
        _check(self.lib.mps_sum_compress_complex(self.h, k, co, re_arr, im_arr, C.byref(dr), C.byref(di), C.byref(o),
                                                 C.byref(stats) if stats is not None else None, _stream()))
        return out_re._written(dr), out_im._written(di)

    def overlap_complex(self, a, b) -> complex:
        """<a|b> of complex states given as (re, im) pairs of DeviceMPS (None = zero part)."""
        r = (C.c_double * 2)()
        descs = [None if m is None else m.desc() for m in (*a, *b)]
        ptrs = [None if d is None else C.byref(d) for d in descs]
        _check(self.lib.mps_overlap_complex(self.h, *ptrs, r, _stream()))
        return complex(r[0], r[1])

    def overlap(self, a: DeviceMPS, b: DeviceMPS) -> float:
        r = C.c_double()
        ad, bd = a.desc(), b.desc()
        _check(self.lib.mps_overlap(self.h, C.byref(ad), C.byref(bd), C.byref(r), _stream()))
        return float(r.value)

    def norm(self, a: DeviceMPS) -> float:
        return float(np.sqrt(max(self.overlap(a, a), 0.0)))


class Krylov:
    """Lanczos state on the device (krylov_create / krylov_step)."""

    def __init__(self, ctx: Context, psi0: DeviceMPS, K: int, D: int, **kw):
        self.ctx = ctx
        self.K = K
        self.opts = make_opts(D, **kw)
        h = C.c_void_p()
        pd = psi0.desc()
        _check(ctx.lib.krylov_create(ctx.h, C.byref(pd), int(K), C.byref(self.opts), C.byref(h), _stream()))
        self.h = h
        self.steps = 0

    def step(self, stats: ThcStats | None = None):
        m = self.steps + 1
        g = (C.c_double * m)()
        t = (C.c_double * m)()
        b = C.c_double()
        _check(self.ctx.lib.krylov_step(self.h, g, t, C.byref(b), C.byref(stats) if stats is not None else None,
                                        _stream()))
        self.steps += 1
        return np.array(g[:]), np.array(t[:]), float(b.value)

    def ritz_vector(self, a: int = 0) -> DeviceMPS:
        """The a-th Ritz vector (ascending Ritz values) of the steps taken."""
        out = DeviceMPS(self.ctx.n, max(capacity(self.ctx.n, self.opts.D_max), 1), self.ctx.device)
        od = out.desc()
        _check(self.ctx.lib.krylov_ritz_vector(self.h, int(a), C.byref(od), _stream()))
        return out._written(od)

    def restart(self, a: int = 0):
        """Restart from the a-th Ritz vector: a new Krylov space of up to K vectors."""
        _check(self.ctx.lib.krylov_restart(self.h, int(a), _stream()))
        self.steps = 0

    def vector(self, i: int, D: int) -> DeviceMPS:
        out = DeviceMPS(self.ctx.n, max(capacity(self.ctx.n, D), 1), self.ctx.device)
        od = out.desc()
        _check(self.ctx.lib.krylov_get_vector(self.h, int(i), C.byref(od), _stream()))
        return out._written(od)

    def matrices(self):
        m = C.c_int32()
        R = self.K + 1
        Mm = (C.c_double * (R * R))()
        S = (C.c_double * (R * R))()
        _check(self.ctx.lib.krylov_get_matrices(self.h, Mm, S, C.byref(m)))
        k = m.value
        return np.array(Mm[: k * k]).reshape(k, k), np.array(S[: k * k]).reshape(k, k)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.krylov_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evolve(instances, K: int, delta: float, n_steps: int, stats: ThcStats | None = None):
    """Krylov time evolution (krylov_evolve) of complex states held as (re, im)
    pairs of DeviceMPS.  instances: list of (Context, re, im, D, opts kw dict)
    with re or im None for a zero part.  Returns ([(re, im), ...] as
    DeviceMPS, krylov basis sizes as an n_inst x n_steps array); a zero part
    comes back as the bond-1 MPS of zeros."""
    q = len(instances)
    lib = load_library()
    ctxs = (C.c_void_p * q)(*[inst[0].h for inst in instances])
    keep = []

    def ptr(m):
        if m is None:
            return None
        d = m.desc()
        keep.append(d)
        return C.pointer(d)

    re_in = (C.POINTER(ThcMps) * q)(*[ptr(inst[1]) for inst in instances])
    im_in = (C.POINTER(ThcMps) * q)(*[ptr(inst[2]) for inst in instances])
    opts = (ThcOpts * q)(*[make_opts(inst[3], **(inst[4] if len(inst) > 4 else {})) for inst in instances])
    outs = []
    for inst in instances:
        ctx, re, im, D = inst[:4]
        cap = capacity(ctx.n, D)
        for m in (re, im):
            if m is not None:
                cap = max(cap, m.buf.numel())
        outs.append((DeviceMPS(ctx.n, cap, ctx.device), DeviceMPS(ctx.n, cap, ctx.device)))
    od = [(a.desc(), b.desc()) for a, b in outs]
    re_out = (C.POINTER(ThcMps) * q)(*[C.pointer(a) for a, _ in od])
    im_out = (C.POINTER(ThcMps) * q)(*[C.pointer(b) for _, b in od])
    dims = (C.c_int32 * max(1, q * n_steps))()
    _check(lib.krylov_evolve(q, ctxs, re_in, im_in, opts, int(K), float(delta), int(n_steps), re_out, im_out, dims,
                             C.byref(stats) if stats is not None else None, _stream()))
    res = [(a._written(da), b._written(db)) for (a, b), (da, db) in zip(outs, od)]
    return res, np.array(dims[: q * n_steps], dtype=np.int32).reshape(q, n_steps)


class ThcEnergy(torch.autograd.Function):
    """E(chi, zeta) = <psi|H|psi> for a fixed MPS psi and one-body t, with the
    hand-written adjoint of thc_energy_gradient as its backward.  chi (L x N)
    and zeta (N x N) are float64 tensors (any device); the factors are loaded
    into a fresh context on every call."""

    @staticmethod
    def forward(fctx, chi, zeta, t, psi, prec="f64"):
        c = Context(np.asarray(t, dtype=np.float64), chi.detach().double().cpu().numpy(),
                    zeta.detach().double().cpu().numpy(), device=psi.buf.device)
        e, dchi, dzeta = c.energy_gradient(psi, prec)
        c.close()
        fctx.save_for_backward(torch.from_numpy(dchi).to(chi.device, chi.dtype),
                               torch.from_numpy(dzeta).to(zeta.device, zeta.dtype))
        return torch.tensor(e, dtype=chi.dtype, device=chi.device)

    @staticmethod
    def backward(fctx, g):
        dchi, dzeta = fctx.saved_tensors
        return g * dchi, g * dzeta, None, None, None


def thc_energy(chi, zeta, t, psi: DeviceMPS, prec="f64"):
    """Differentiable E = <psi|H(t, chi, zeta)|psi> (see ThcEnergy)."""
    return ThcEnergy.apply(chi, zeta, t, psi, prec)
