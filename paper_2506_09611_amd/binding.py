"""ctypes binding of libpqmc.so (include/pqmc.h), same names as the C ABI.

Argument marshalling only: every step of the sweep runs in the library's
HIP kernels.  The device workspace is one torch uint8 tensor on the
current CUDA (HIP) device and work goes to torch's current stream.
"""
from __future__ import annotations

import ctypes
import enum
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

EXPORTED_SYMBOLS = (
    "pqmc_workspace_bytes", "pqmc_create", "pqmc_set_opts", "pqmc_set_fields",
    "pqmc_get_fields", "pqmc_sweep", "pqmc_forward_window", "pqmc_batch_sweep",
    "pqmc_batch_forward_window", "pqmc_multi_sweep", "pqmc_get_green",
    "pqmc_get_decisions", "pqmc_get_heat_bath", "pqmc_get_kernel_times", "pqmc_destroy",
    "pqmc_replay", "pqmc_get_green_static",
    "pqmc_last_error",
    "pqmc_soc_workspace_bytes", "pqmc_soc_create", "pqmc_soc_sweep", "pqmc_soc_forward_window",
    "pqmc_soc_get_green", "pqmc_soc_get_fields", "pqmc_soc_get_decisions", "pqmc_soc_destroy",
    "pqmc_soc_batch_sweep", "pqmc_soc_batch_forward_window",
)
KERNEL_CLASSES = ("propagate", "local", "tile", "reduce", "decide")


class Scheme(enum.IntEnum):
    LOCAL = 0
    DELAYED = 1
    BLOCK_FB = 2
    LOCAL_G = 3


FLAG_LOG = 1
FLAG_TIMING = 2
FLAG_KTIME = 4
FLAG_FP32 = 8
FLAG_SITE_LAUNCHES = 16
FLAG_GRAPH = 32
FLAG_DENSE_PROP = 64


class PQMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pqmc status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("hopping", ctypes.POINTER(ctypes.c_double)),
                ("trial_up", ctypes.POINTER(ctypes.c_double)),
                ("trial_dn", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_double), ("dtau", ctypes.c_double),
                ("n_slices", ctypes.c_int32), ("stab_every", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("walker_id", ctypes.c_uint64)]


class SocProblem(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_e", ctypes.c_int32),
                ("hopping", ctypes.POINTER(ctypes.c_double)),
                ("trial", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.c_double), ("dtau", ctypes.c_double),
                ("n_slices", ctypes.c_int32), ("stab_every", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("walker_id", ctypes.c_uint64)]


class UpdateOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("delay_k", ctypes.c_int32),
                ("block_b", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("tile_chunks", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("proposed", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("flips", ctypes.c_uint64), ("low_margin", ctypes.c_uint64),
                ("negative", ctypes.c_uint64), ("field_updates", ctypes.c_uint64),
                ("t_total_s", ctypes.c_double), ("t_update_s", ctypes.c_double),
                ("t_prop_s", ctypes.c_double), ("t_stab_s", ctypes.c_double),
                ("max_stab_drift", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def library_path() -> str:
    return os.path.join(_HERE, "libpqmc.so")


def load_library():
    """Load the in-tree libpqmc.so; raise ImportError if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    c_void_p, c_size_t = ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "pqmc_workspace_bytes": [ctypes.POINTER(Problem), ctypes.POINTER(UpdateOpts),
                                 ctypes.POINTER(c_size_t)],
        "pqmc_create": [ctypes.POINTER(Problem), ctypes.POINTER(UpdateOpts), c_void_p, c_void_p,
                        c_size_t, ctypes.POINTER(c_void_p)],
        "pqmc_set_opts": [c_void_p, ctypes.POINTER(UpdateOpts)],
        "pqmc_set_fields": [c_void_p, ctypes.POINTER(ctypes.c_int8)],
        "pqmc_get_fields": [c_void_p, ctypes.POINTER(ctypes.c_int8)],
        "pqmc_sweep": [c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)],
        "pqmc_forward_window": [c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)],
        "pqmc_batch_sweep": [ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(Stats)],
        "pqmc_batch_forward_window": [ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(Stats)],
        "pqmc_multi_sweep": [ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(Stats)],
        "pqmc_get_green": [c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
        "pqmc_get_decisions": [c_void_p, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double), c_size_t,
                               ctypes.POINTER(c_size_t)],
        "pqmc_get_heat_bath": [c_void_p, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double), c_size_t,
                               ctypes.POINTER(c_size_t)],
        "pqmc_get_kernel_times": [c_void_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_uint64)],
        "pqmc_destroy": [c_void_p],
        "pqmc_replay": [c_void_p, ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(Stats)],
        "pqmc_get_green_static": [c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
        "pqmc_soc_workspace_bytes": [ctypes.POINTER(SocProblem), ctypes.POINTER(UpdateOpts),
                                     ctypes.POINTER(c_size_t)],
        "pqmc_soc_create": [ctypes.POINTER(SocProblem), ctypes.POINTER(UpdateOpts), c_void_p,
                            c_void_p, c_size_t, ctypes.POINTER(c_void_p)],
        "pqmc_soc_sweep": [c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)],
        "pqmc_soc_forward_window": [c_void_p, ctypes.c_int32, ctypes.POINTER(Stats)],
        "pqmc_soc_get_green": [c_void_p, ctypes.POINTER(ctypes.c_double)],
        "pqmc_soc_get_fields": [c_void_p, ctypes.POINTER(ctypes.c_int8)],
        "pqmc_soc_get_decisions": [c_void_p, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_double), c_size_t,
                                   ctypes.POINTER(c_size_t)],
        "pqmc_soc_destroy": [c_void_p],
        "pqmc_soc_batch_sweep": [ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(Stats)],
        "pqmc_soc_batch_forward_window": [ctypes.POINTER(c_void_p), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.POINTER(Stats)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pqmc_last_error.argtypes = []
    lib.pqmc_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(lib, status):
    if status != 0:
        raise PQMCError(status, lib.pqmc_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Chain:
    """One PQMC walker on the GPU (a pqmc_ctx).

    hopping: N x N float64; trial_up/trial_dn: N x N_s float64 (orthonormal
    columns); U (U < 0: one complex sector, G complex); dtau; n_slices = M;
    stab_every = k_tau; seed, walker_id:
    Philox key.  scheme / k / b: update scheme, delay rank, block size; k_max
    and b_max bound later set_opts calls (workspace sizing).  stream: the
    torch.cuda.Stream the walker's work goes to (default: the current one);
    the workspace is allocated on it.  tile_chunks: column chunks per row
    strip of the fused flush kernel (0: two, for batches; a large value: one
    tile per workgroup, for a walker run alone).  dense_prop: propagate
    with the dense K = e^{-dtau H0} (GEMMs) even when H0 is sparse enough
    for the Taylor-series propagation (the default where it applies).
    """

    def __init__(self, hopping, trial_up, trial_dn, U, dtau, n_slices, stab_every, seed,
                 walker_id=0, scheme=Scheme.LOCAL, k=1, b=1, k_max=None, b_max=None,
                 log=False, timing=False, fp32=False, stream=None, tile_chunks=0,
                 dense_prop=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self._lib = load_library()
        self._H = np.ascontiguousarray(hopping, dtype=np.float64)
        self._Pu = np.ascontiguousarray(trial_up, dtype=np.float64)
        self._Pd = np.ascontiguousarray(trial_dn, dtype=np.float64)
        N = self._H.shape[0]
        self.N, self.M = N, int(n_slices)
        # U < 0: the paper's one complex sector (spin down = its conjugate)
        self.complex = float(U) < 0
        self.n_up, self.n_dn = self._Pu.shape[1], self._Pd.shape[1]
        self._prob = Problem(N, self.n_up, self.n_dn, _dptr(self._H), _dptr(self._Pu),
                             _dptr(self._Pd), float(U), float(dtau), int(n_slices),
                             int(stab_every), int(seed) & (2**64 - 1), int(walker_id))
        self._flags = ((FLAG_LOG if log else 0) | (FLAG_TIMING if timing else 0)
                       | (FLAG_FP32 if fp32 else 0) | (FLAG_DENSE_PROP if dense_prop else 0))
        kmax = int(k_max if k_max is not None else k)
        bmax = int(b_max if b_max is not None else b)
        self.tile_chunks = int(tile_chunks)
        sizing = UpdateOpts(int(scheme), max(kmax, 1), max(bmax, 1), self._flags,
                            self.tile_chunks)
        nbytes = ctypes.c_size_t(0)
        _check(self._lib, self._lib.pqmc_workspace_bytes(ctypes.byref(self._prob),
                                                         ctypes.byref(sizing),
                                                         ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(self._stream):
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        base = (base + 255) // 256 * 256
        handle = ctypes.c_void_p(0)
        _check(self._lib, self._lib.pqmc_create(ctypes.byref(self._prob), ctypes.byref(sizing),
                                                ctypes.c_void_p(self._stream.cuda_stream),
                                                ctypes.c_void_p(base),
                                                ctypes.c_size_t(nbytes.value),
                                                ctypes.byref(handle)))
        self._ctx = handle
        self.set_opts(scheme, k, b)

    # -- calls with the C ABI's names
    def set_opts(self, scheme, k=1, b=1, log=None, timing=None, ktime=None, fp32=None,
                 tile_chunks=None, site_launches=None, graph=None, dense_prop=None):
        flags = self._flags
        if dense_prop is not None:
            flags = (flags & ~FLAG_DENSE_PROP) | (FLAG_DENSE_PROP if dense_prop else 0)
        if graph is not None:
            flags = (flags & ~FLAG_GRAPH) | (FLAG_GRAPH if graph else 0)
        if site_launches is not None:
            flags = (flags & ~FLAG_SITE_LAUNCHES) | (FLAG_SITE_LAUNCHES if site_launches else 0)
        if tile_chunks is not None:
            self.tile_chunks = int(tile_chunks)
        if fp32 is not None:
            flags = (flags & ~FLAG_FP32) | (FLAG_FP32 if fp32 else 0)
        if ktime is not None:
            flags = (flags & ~FLAG_KTIME) | (FLAG_KTIME if ktime else 0)
        if log is not None:
            flags = (flags & ~FLAG_LOG) | (FLAG_LOG if log else 0)
        if timing is not None:
            flags = (flags & ~FLAG_TIMING) | (FLAG_TIMING if timing else 0)
        o = UpdateOpts(int(scheme), int(k), int(b), flags, self.tile_chunks)
        _check(self._lib, self._lib.pqmc_set_opts(self._ctx, ctypes.byref(o)))
        self.scheme, self.k, self.b, self._flags = Scheme(int(scheme)), int(k), int(b), flags

    def sweep(self, n=1):
        st = Stats()
        _check(self._lib, self._lib.pqmc_sweep(self._ctx, int(n), ctypes.byref(st)))
        return st.as_dict()

    def forward_window(self, n_slices):
        st = Stats()
        _check(self._lib, self._lib.pqmc_forward_window(self._ctx, int(n_slices),
                                                        ctypes.byref(st)))
        return st.as_dict()

    def replay(self, flips):
        """pqmc_replay: one sweep with every outcome forced by flips (2M x N,
        nonzero = the site's field flips on that slice visit)."""
        f = np.ascontiguousarray(flips, dtype=np.int8).reshape(2 * self.M, self.N)
        st = Stats()
        _check(self._lib, self._lib.pqmc_replay(
            self._ctx, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), ctypes.byref(st)))
        return st.as_dict()

    def green(self, spin):
        """G of the spin sector (N x N); complex128 when U < 0."""
        out = np.empty((self.N, self.N), np.complex128 if self.complex else np.float64)
        _check(self._lib, self._lib.pqmc_get_green(
            self._ctx, int(spin), out.view(np.float64).ctypes.data_as(
                ctypes.POINTER(ctypes.c_double))))
        return out

    def fields(self):
        out = np.empty((self.M, self.N), np.int8)
        _check(self._lib, self._lib.pqmc_get_fields(
            self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def set_fields(self, fields):
        f = np.ascontiguousarray(fields, dtype=np.int8).reshape(self.M, self.N)
        _check(self._lib, self._lib.pqmc_set_fields(
            self._ctx, f.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))

    def _log(self, fn):
        n = ctypes.c_size_t(0)
        _check(self._lib, fn(self._ctx, None, None, 0, ctypes.byref(n)))
        meta = np.empty((max(n.value, 1), 3), np.int32)
        margin = np.empty(max(n.value, 1), np.float64)
        _check(self._lib, fn(self._ctx, meta.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             _dptr(margin), n.value, ctypes.byref(n)))
        return meta[:n.value], margin[:n.value]

    def decisions(self):
        """(meta[n, 3] = (dir*M + l-1, site, accepted), margin[n]) of the last call."""
        return self._log(self._lib.pqmc_get_decisions)

    def heat_bath(self):
        return self._log(self._lib.pqmc_get_heat_bath)

    def kernel_times(self):
        """{class: (total_seconds, launches)} of the last call made with ktime on."""
        tot = (ctypes.c_double * len(KERNEL_CLASSES))()
        cnt = (ctypes.c_uint64 * len(KERNEL_CLASSES))()
        _check(self._lib, self._lib.pqmc_get_kernel_times(self._ctx, tot, cnt))
        return {k: (tot[i], int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def close(self):
        """Destroy the context and release its workspace (to torch's caching
        allocator, stream-ordered, so work already queued is unaffected)."""
        if getattr(self, "_ctx", None):
            self._lib.pqmc_destroy(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def soc_workspace_bytes(n_sites, n_e, n_slices, stab_every, scheme=Scheme.DELAYED, k=16,
                        log=False):
    """pqmc_soc_workspace_bytes for an SOC problem of this shape (+256 bytes
    of alignment slack): the whole device footprint of one SocChain."""
    lib = load_library()
    n2 = 2 * int(n_sites)
    z = np.zeros((n2, n2), np.complex128)
    pt = np.zeros((n2, int(n_e)), np.complex128)
    prob = SocProblem(int(n_sites), int(n_e), z.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), pt.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), -1.0, 0.05, int(n_slices), int(stab_every), 0, 0)
    o = UpdateOpts(int(scheme), max(int(k), 1), max(int(k), 1), FLAG_LOG if log else 0)
    n = ctypes.c_size_t(0)
    _check(lib, lib.pqmc_soc_workspace_bytes(ctypes.byref(prob), ctypes.byref(o),
                                             ctypes.byref(n)))
    return n.value + 256


class SocChain:
    """One walker of the spin-orbit coupled Hubbard model (a pqmc_soc_ctx).

    hopping: 2N x 2N complex128 Hermitian (basis c_1up..c_Nup, c_1dn..c_Ndn);
    trial: 2N x N_e complex128 with orthonormal columns; U <= 0; scheme
    LOCAL, DELAYED (k sites per flush) or BLOCK_FB (blocks of k sites); k <= 32.
    """

    def __init__(self, hopping, trial, U, dtau, n_slices, stab_every, seed, walker_id=0,
                 scheme=Scheme.DELAYED, k=16, log=False, timing=False, stream=None,
                 dense_prop=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self._lib = load_library()
        self._H = np.ascontiguousarray(hopping, dtype=np.complex128)
        self._P = np.ascontiguousarray(trial, dtype=np.complex128)
        n2 = self._H.shape[0]
        self.N, self.M, self.n_e = n2 // 2, int(n_slices), self._P.shape[1]
        self._prob = SocProblem(self.N, self.n_e, self._H.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), self._P.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), float(U), float(dtau), int(n_slices),
            int(stab_every), int(seed) & (2**64 - 1), int(walker_id))
        flags = ((FLAG_LOG if log else 0) | (FLAG_TIMING if timing else 0)
                 | (FLAG_DENSE_PROP if dense_prop else 0))
        self._opts = UpdateOpts(int(scheme), int(k), int(k), flags)
        nbytes = ctypes.c_size_t(0)
        _check(self._lib, self._lib.pqmc_soc_workspace_bytes(
            ctypes.byref(self._prob), ctypes.byref(self._opts), ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(self._stream):
            self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = (self._ws.data_ptr() + 255) // 256 * 256
        handle = ctypes.c_void_p(0)
        _check(self._lib, self._lib.pqmc_soc_create(
            ctypes.byref(self._prob), ctypes.byref(self._opts),
            ctypes.c_void_p(self._stream.cuda_stream), ctypes.c_void_p(base),
            ctypes.c_size_t(nbytes.value), ctypes.byref(handle)))
        self._ctx = handle
        self.scheme, self.k = Scheme(int(scheme)), int(k)

    def sweep(self, n=1):
        st = Stats()
        _check(self._lib, self._lib.pqmc_soc_sweep(self._ctx, int(n), ctypes.byref(st)))
        return st.as_dict()

    def forward_window(self, n_slices):
        st = Stats()
        _check(self._lib, self._lib.pqmc_soc_forward_window(self._ctx, int(n_slices),
                                                            ctypes.byref(st)))
        return st.as_dict()

    def green(self):
        out = np.empty((2 * self.N, 2 * self.N), np.complex128)
        _check(self._lib, self._lib.pqmc_soc_get_green(
            self._ctx, out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def fields(self):
        out = np.empty((self.M, self.N), np.int8)
        _check(self._lib, self._lib.pqmc_soc_get_fields(
            self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def decisions(self):
        """(meta[n, 3] = (dir*M + l-1, site, accepted), margin[n]) of the last call."""
        fn = self._lib.pqmc_soc_get_decisions
        n = ctypes.c_size_t(0)
        _check(self._lib, fn(self._ctx, None, None, 0, ctypes.byref(n)))
        meta = np.empty((max(n.value, 1), 3), np.int32)
        margin = np.empty(max(n.value, 1), np.float64)
        _check(self._lib, fn(self._ctx, meta.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             _dptr(margin), n.value, ctypes.byref(n)))
        return meta[:n.value], margin[:n.value]

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pqmc_soc_destroy(self._ctx)
            self._ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MAX_BATCH = 8


def workspace_bytes(n_sites, n_up, n_dn, n_slices, stab_every, scheme=Scheme.DELAYED, k=1,
                    b=1, fp32=False, log=False):
    """pqmc_workspace_bytes for a problem of this shape: the whole device
    footprint of one Chain (the library allocates nothing else), +256 bytes
    of alignment slack.  Needs the library but no GPU."""
    lib = load_library()
    z = np.zeros((n_sites, n_sites))
    pu, pd = np.zeros((n_sites, n_up)), np.zeros((n_sites, n_dn))
    prob = Problem(int(n_sites), int(n_up), int(n_dn), _dptr(z), _dptr(pu), _dptr(pd), 0.0,
                   0.05, int(n_slices), int(stab_every), 0, 0)
    flags = (FLAG_FP32 if fp32 else 0) | (FLAG_LOG if log else 0)
    o = UpdateOpts(int(scheme), max(int(k), 1), max(int(b), 1), flags)
    n = ctypes.c_size_t(0)
    _check(lib, lib.pqmc_workspace_bytes(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(n)))
    return n.value + 256


def _batch_call(chains, fn, n, limit=MAX_BATCH):
    if not 1 <= len(chains) <= limit:
        raise ValueError(f"a batch holds 1..{limit} chains")
    lib = chains[0]._lib
    ctxs = (ctypes.c_void_p * len(chains))(*[c._ctx.value for c in chains])
    st = (Stats * len(chains))()
    _check(lib, fn(lib)(ctxs, len(chains), int(n), st))
    return [s.as_dict() for s in st]


def batch_sweep(chains, n=1):
    """pqmc_batch_sweep: n sweeps of up to 8 chains in lockstep, one launch
    per kernel for all of them (the delayed and block schemes accept chains of
    different lattice sizes).  Returns one stats dict per chain."""
    return _batch_call(chains, lambda lib: lib.pqmc_batch_sweep, n)


def multi_sweep(chains, n=1):
    """pqmc_multi_sweep: up to 128 chains on up to 16 streams; the chains of
    one stream sweep as one batch and the batches run concurrently."""
    if not 1 <= len(chains) <= 16 * MAX_BATCH:
        raise ValueError(f"a multi-stream sweep holds 1..{16 * MAX_BATCH} chains")
    return _batch_call(chains, lambda lib: lib.pqmc_multi_sweep, n, limit=16 * MAX_BATCH)


def batch_forward_window(chains, n_slices):
    """pqmc_batch_forward_window for up to 8 chains (rules of batch_sweep)."""
    return _batch_call(chains, lambda lib: lib.pqmc_batch_forward_window, n_slices)


def soc_batch_sweep(chains, n=1):
    """pqmc_soc_batch_sweep: n sweeps of up to 8 SocChains of one lattice,
    N_e, M, k_tau, scheme, k and stream in lockstep (one launch per kernel for
    all of them).  Returns one stats dict per chain."""
    return _batch_call(chains, lambda lib: lib.pqmc_soc_batch_sweep, n)


def soc_batch_forward_window(chains, n_slices):
    """pqmc_soc_batch_forward_window for up to 8 SocChains (rules of
    soc_batch_sweep)."""
    return _batch_call(chains, lambda lib: lib.pqmc_soc_batch_forward_window, n_slices)
