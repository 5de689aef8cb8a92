"""ctypes binding of libcpra.so (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; PyTorch is
used here only to own device memory (the plan workspace, inputs, outputs)
and to supply the HIP stream.  There is no CPU fallback: if the library is
missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpra.so")

CPRA_OK = 0
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_OOM", -3: "ERR_DEVICE", -4: "ERR_STATE", -5: "ERR_UNSUPPORTED",
          -6: "ERR_DATA"}
HIO, ER, RAAR = 0, 1, 2
INSERT_NEAREST, INSERT_BILINEAR = 0, 1
WRAP_MIRROR, WRAP_PLAIN = 0, 1
REAL_F32, REAL_F64 = 0, 1
AMP_F32, AMP_F16 = 0, 1
PTR_HOST, PTR_DEVICE, PTR_DEVICE_ASYNC = 0, 1, 2

EXPORTED = [
    "cpra_workspace_size", "cpra_plan", "cpra_plan_create", "cpra_submit_angles", "cpra_iterate", "cpra_read_objects",
    "cpra_assemble_volume", "cpra_destroy", "cpra_last_error", "cpra_iteration_count", "cpra_slice_cells",
    "cpra_coupling_table", "cpra_set_kernel_timing", "cpra_kernel_timing", "cpra_load_objects",
    "cpra_iterate_batch", "cpra_prereconstruct", "cpra_sweep", "cpra_merge", "cpra_shrinkwrap",
    "cpra_read_support", "cpra_refine_workspace_size", "cpra_refine_volume", "cpra_set_graphs", "cpra_set_chunk",
    "cpra_refine_volume_noalloc", "cpra_set_batch_fusion", "cpra_get_batch_fusion", "cpra_set_tuning",
    "cpra_autotune",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("N", ctypes.c_int32),
        ("Np", ctypes.c_int32),
        ("theta", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.c_double * 3),
        ("n_ei", ctypes.c_int32),
        ("wrap", ctypes.c_int32),
        ("positivity", ctypes.c_int32),
        ("real_type", ctypes.c_int32),
        ("amp_type", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("n_guess", ctypes.c_int32),
        ("insertion", ctypes.c_int32),
        ("taps", ctypes.POINTER(ctypes.c_double)),
        ("n_taps", ctypes.c_int32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("row_tile", ctypes.c_int32), ("chunk", ctypes.c_int32), ("graphs", ctypes.c_int32),
                ("ms_per_iteration", ctypes.c_double)]

    def as_dict(self):
        return {"row_tile": self.row_tile, "chunk": self.chunk, "graphs": self.graphs,
                "ms_per_iteration": self.ms_per_iteration}


class CpraError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libcpra.so (built in-tree by paper_2402_05283_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2402_05283_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P = c.POINTER
    lib.cpra_workspace_size.argtypes = [P(Params), P(c.c_size_t)]
    lib.cpra_plan.argtypes = [P(Params), c.c_void_p, c.c_size_t, c.c_void_p, P(c.c_void_p)]
    lib.cpra_plan_create.argtypes = [P(Params), c.c_void_p, c.c_size_t, c.c_void_p, P(c.c_void_p)]
    lib.cpra_submit_angles.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_void_p, c.c_void_p, c.c_int32]
    lib.cpra_iterate.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_double, c.c_void_p]
    lib.cpra_read_objects.argtypes = [c.c_void_p, c.c_void_p, c.c_int32]
    lib.cpra_assemble_volume.argtypes = [c.c_void_p, c.c_void_p]
    lib.cpra_destroy.argtypes = [c.c_void_p]
    lib.cpra_iterate_batch.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_int32, c.c_double]
    lib.cpra_prereconstruct.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_double, c.c_void_p]
    lib.cpra_sweep.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_double, c.c_void_p]
    lib.cpra_merge.argtypes = [c.c_void_p, c.c_int32, c.c_void_p, c.c_void_p]
    lib.cpra_shrinkwrap.argtypes = [c.c_void_p, c.c_double, c.c_double]
    lib.cpra_read_support.argtypes = [c.c_void_p, c.c_void_p]
    lib.cpra_set_graphs.argtypes = [c.c_void_p, c.c_int32]
    lib.cpra_set_chunk.argtypes = [c.c_void_p, c.c_int32]
    lib.cpra_refine_workspace_size.argtypes = [P(Params), P(c.c_size_t)]
    lib.cpra_refine_volume.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_double, c.c_double, c.c_void_p,
                                       c.c_size_t, c.c_void_p]
    lib.cpra_refine_volume_noalloc.argtypes = [c.c_void_p, c.c_int32, c.c_int32, c.c_double, c.c_double,
                                               c.c_void_p]
    lib.cpra_set_batch_fusion.argtypes = [c.c_int32]
    lib.cpra_set_tuning.argtypes = [c.c_void_p, P(Tuning)]
    lib.cpra_autotune.argtypes = [P(Params), c.c_void_p, c.c_size_t, c.c_void_p, c.c_int32, P(Tuning)]
    lib.cpra_get_batch_fusion.argtypes = [P(c.c_int32)]
    lib.cpra_last_error.argtypes = [c.c_void_p]
    lib.cpra_last_error.restype = c.c_char_p
    lib.cpra_iteration_count.argtypes = [c.c_void_p, P(c.c_int64)]
    lib.cpra_slice_cells.argtypes = [c.c_int32, c.c_int32, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.cpra_coupling_table.argtypes = [P(Params), c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.cpra_load_objects.argtypes = [c.c_void_p, c.c_void_p, c.c_int32]
    lib.cpra_set_kernel_timing.argtypes = [c.c_void_p, c.c_int32]
    lib.cpra_kernel_timing.argtypes = [c.c_void_p, P(c.c_double), P(c.c_int64), P(c.c_double), P(c.c_int64)]
    for name in EXPORTED:
        if name != "cpra_last_error":
            getattr(lib, name).restype = c.c_int
    _lib = lib
    return lib


def _check(st, plan=None):
    if st != CPRA_OK:
        msg = load().cpra_last_error(plan)
        raise CpraError(st, msg.decode() if msg else "")


def autotune(N, Np, n_iter=20, stream=None, **kw):
    """cpra_autotune on a temporary workspace: the fastest launch choices for plans of this shape
    (recorded in the library for plans created afterwards); returns them as a dict."""
    import torch
    p = make_params(N, Np, **kw)
    nbytes = workspace_size(p)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) // 256 * 256
    st = torch.cuda.current_stream() if stream is None else stream
    best = Tuning()
    _check(load().cpra_autotune(ctypes.byref(p), ctypes.c_void_p(ptr), nbytes, ctypes.c_void_p(st.cuda_stream),
                                int(n_iter), ctypes.byref(best)))
    del ws
    return best.as_dict()


def get_batch_fusion():
    """cpra_get_batch_fusion: the size limit of shared launches in iterate_batch."""
    v = ctypes.c_int32(0)
    _check(load().cpra_get_batch_fusion(ctypes.byref(v)))
    return v.value


def set_batch_fusion(max_n):
    """cpra_set_batch_fusion: plans of one size class with N <= max_n share launches in
    iterate_batch (0: none).  Returns the previous setting."""
    prev = ctypes.c_int32(0)
    _check(load().cpra_get_batch_fusion(ctypes.byref(prev)))
    _check(load().cpra_set_batch_fusion(int(max_n)))
    return prev.value


def iterate_batch(plans, n_iter, algo=HIO, beta=0.9):
    """cpra_iterate_batch over a list of Plan objects (each on its own stream, ideally)."""
    handles = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    st = load().cpra_iterate_batch(handles, len(plans), int(n_iter), int(algo), float(beta))
    if st != CPRA_OK:
        msgs = [load().cpra_last_error(p.handle) for p in plans] + [load().cpra_last_error(None)]
        raise CpraError(st, "; ".join(m.decode() for m in msgs if m))


def make_params(N, Np, theta=None, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=WRAP_MIRROR, positivity=True,
                real=REAL_F32, amp=AMP_F32, seed=0, n_guess=1, insertion=0, taps=None):
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    p.N, p.Np = int(N), int(Np)
    p._theta_keep = None
    if theta is not None:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        p._theta_keep = th
        p.theta = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for i in range(3):
        p.alpha[i] = float(alpha[i])
    p.n_ei, p.wrap, p.positivity = int(n_ei), int(wrap), int(bool(positivity))
    p.real_type, p.amp_type = int(real), int(amp)
    p.seed = int(seed) % (1 << 64)
    p.n_guess = int(n_guess)
    p.insertion = int(insertion)
    p._taps_keep = None
    if taps is not None:
        tp = np.ascontiguousarray(taps, dtype=np.float64)
        p._taps_keep = tp
        p.taps = tp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.n_taps = len(tp)
    return p


def workspace_size(params) -> int:
    n = ctypes.c_size_t(0)
    _check(load().cpra_workspace_size(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def slice_cells(N, Np, theta=None):
    kx = np.zeros((Np, N), np.int32)
    ky = np.zeros((Np, N), np.int32)
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
    _check(load().cpra_slice_cells(N, Np, None if th is None else th.ctypes.data, kx.ctypes.data, ky.ctypes.data))
    return kx, ky


def coupling_table(params, present=None):
    Np = params.Np
    left = np.zeros(Np, np.int32)
    right = np.zeros(Np, np.int32)
    w = np.zeros((Np, 3), np.float64)
    mirror = np.zeros((Np, 2), np.uint8)
    pr = None if present is None else np.ascontiguousarray(present, dtype=np.uint8)
    _check(load().cpra_coupling_table(ctypes.byref(params), None if pr is None else pr.ctypes.data, left.ctypes.data,
                                      right.ctypes.data, w.ctypes.data, mirror.ctypes.data))
    return left, right, w, mirror


class Plan:
    """One scan on the current device: owns a torch workspace tensor and a library plan."""

    def __init__(self, N, Np, theta=None, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=WRAP_MIRROR, positivity=True,
                 real=REAL_F32, amp=AMP_F32, seed=0, stream=None, device=None, n_guess=1, insertion=0,
                 taps=None):
        import torch
        self.torch = torch
        lib = load()
        self.params = make_params(N, Np, theta, alpha, n_ei, wrap, positivity, real, amp, seed, n_guess, insertion,
                                  taps)
        self.N, self.Np = int(N), int(Np)
        self.R = max(1, int(n_guess))
        self.real = real
        self.dtype = torch.float64 if real == REAL_F64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = workspace_size(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        handle = ctypes.c_void_p(0)
        self._pid = os.getpid()
        st = lib.cpra_plan(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle))
        _check(st, None)
        self.handle = handle

    def _enter(self):
        """Order the plan's stream after the caller's current stream (tensors handed in were
        produced there)."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self, *tensors):
        """Order the caller's current stream after the plan's stream, and keep tensors the
        library touched alive for the plan's stream."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
            for t in tensors:
                t.record_stream(self.stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        # a forked child process (a worker pool) holds a copy of the object but not the GPU state:
        # only the creating process destroys the plan
        if h is not None and h.value and getattr(self, "_pid", None) == os.getpid():
            load().cpra_destroy(h)
            self.handle = None

    def submit(self, first, intensity, support, asynchronous=False):
        """intensity: (count,N,N) float32; support: (count,N,N) uint8 — torch CUDA tensors or numpy arrays.
        asynchronous (CUDA tensors): the library does not wait for the GPU; a NaN/Inf in the
        intensities is reported by a later call (and poisons the plan); the tensors are kept alive
        for the plan's stream."""
        torch = self.torch
        if isinstance(intensity, np.ndarray):
            I = np.ascontiguousarray(intensity, dtype=np.float32)
            S = np.ascontiguousarray(support, dtype=np.uint8)
            count = I.shape[0]
            st = load().cpra_submit_angles(self.handle, first, count, I.ctypes.data, S.ctypes.data, PTR_HOST)
        else:
            I = intensity.contiguous()
            S = support.contiguous()
            if I.dtype != torch.float32 or S.dtype != torch.uint8 or not I.is_cuda or not S.is_cuda:
                raise TypeError("device inputs must be CUDA float32 intensity and uint8 support")
            count = I.shape[0]
            self._enter()       # the library reads I and S on its stream
            st = load().cpra_submit_angles(self.handle, first, count, ctypes.c_void_p(I.data_ptr()),
                                           ctypes.c_void_p(S.data_ptr()), PTR_DEVICE_ASYNC if asynchronous else PTR_DEVICE)
            if asynchronous and st == CPRA_OK:
                self._leave(I, S)
        _check(st, self.handle)

    def iterate(self, n_iter, algo=HIO, beta=0.9, errors=False):
        """Jacobi step B; returns E_F (n_iter, Np), or (n_iter, n_guess * Np) for several guesses."""
        err = np.zeros((n_iter, self.R * self.Np), np.float64) if errors else None
        st = load().cpra_iterate(self.handle, int(n_iter), int(algo), float(beta),
                                 None if err is None else err.ctypes.data)
        _check(st, self.handle)
        return err

    def _obj_shape(self):
        return (self.Np, self.N, self.N) if self.R == 1 else (self.R, self.Np, self.N, self.N)

    def prereconstruct(self, n_iter, algo=HIO, beta=0.9, errors=False):
        """Step A on angle 0 of every guess; returns E_F (n_guess, n_iter) if errors."""
        err = np.zeros((self.R, n_iter), np.float64) if errors else None
        _check(load().cpra_prereconstruct(self.handle, int(n_iter), int(algo), float(beta),
                                          None if err is None else err.ctypes.data), self.handle)
        return err

    def sweep(self, n_episodes, algo=HIO, beta=0.9, errors=False):
        """Consecutive step B; returns E_F (n_episodes, n_guess, Np, n_ei) if errors."""
        err = np.zeros((n_episodes, self.R, self.Np, self.params.n_ei), np.float64) if errors else None
        _check(load().cpra_sweep(self.handle, int(n_episodes), int(algo), float(beta),
                                 None if err is None else err.ctypes.data), self.handle)
        return err

    def merge(self, n_best):
        """Step C; returns (kept guesses in rank order, inverted flags)."""
        kept = np.zeros(n_best, np.int32)
        inv = np.zeros(n_best, np.int32)
        _check(load().cpra_merge(self.handle, int(n_best), kept.ctypes.data, inv.ctypes.data), self.handle)
        return kept, inv.astype(bool)

    def shrinkwrap(self, sigma, threshold):
        """Replace every present angle's support by the shrinkwrap of its current object."""
        _check(load().cpra_shrinkwrap(self.handle, float(sigma), float(threshold)), self.handle)

    def refine_volume(self, n_iter, shrink_every=0, sigma=1.0, threshold=0.1, out=None):
        """3D refinement after step D; returns the refined (N, N, N) volume."""
        torch = self.torch
        n = ctypes.c_size_t(0)
        _check(load().cpra_refine_workspace_size(ctypes.byref(self.params), ctypes.byref(n)))
        work = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        wp = (work.data_ptr() + 255) // 256 * 256
        if out is None:
            out = torch.empty((self.N, self.N, self.N), dtype=self.dtype, device=self.device)
        self._enter()
        _check(load().cpra_refine_volume(self.handle, int(n_iter), int(shrink_every), float(sigma), float(threshold),
                                         ctypes.c_void_p(wp), n.value, ctypes.c_void_p(out.data_ptr())), self.handle)
        self._leave(out, work)
        return out

    def refine_volume_noalloc(self, n_iter, out, shrink_every=0, sigma=1.0, threshold=0.1):
        """cpra_refine_volume_noalloc into the caller's (N, N, N) volume `out` (no device allocation
        here or in the library)."""
        self._enter()
        _check(load().cpra_refine_volume_noalloc(self.handle, int(n_iter), int(shrink_every), float(sigma),
                                                 float(threshold), ctypes.c_void_p(out.data_ptr())), self.handle)
        self._leave(out)
        return out

    def support(self):
        """The supports in use, (Np, N, N) uint8 (host)."""
        out = np.zeros((self.Np, self.N, self.N), np.uint8)
        _check(load().cpra_read_support(self.handle, out.ctypes.data), self.handle)
        return out

    def objects(self, out=None):
        """Current iterates: (Np, N, N), or (n_guess, Np, N, N) for several guesses."""
        torch = self.torch
        if out is None:
            out = torch.empty(self._obj_shape(), dtype=self.dtype, device=self.device)
        self._enter()
        _check(load().cpra_read_objects(self.handle, ctypes.c_void_p(out.data_ptr()), PTR_DEVICE), self.handle)
        self._leave(out)
        return out

    def load_objects(self, objects):
        """Warm start: set the current iterate of every submitted angle (torch CUDA tensor or numpy array)."""
        torch = self.torch
        if isinstance(objects, np.ndarray):
            a = np.ascontiguousarray(objects, dtype=np.float64 if self.real == REAL_F64 else np.float32)
            if a.shape != self._obj_shape():
                raise ValueError(f"objects must be {self._obj_shape()}")
            st = load().cpra_load_objects(self.handle, a.ctypes.data, PTR_HOST)
        else:
            a = objects.contiguous()
            if a.dtype != self.dtype or tuple(a.shape) != self._obj_shape() or not a.is_cuda:
                raise TypeError(f"objects must be a CUDA tensor of shape {self._obj_shape()} in the plan's precision")
            self._enter()       # synchronises before returning
            st = load().cpra_load_objects(self.handle, ctypes.c_void_p(a.data_ptr()), PTR_DEVICE)
        _check(st, self.handle)

    def assemble_volume(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty((self.N, self.N, self.N), dtype=self.dtype, device=self.device)
        self._enter()
        _check(load().cpra_assemble_volume(self.handle, ctypes.c_void_p(out.data_ptr())), self.handle)
        self._leave(out)
        return out

    def set_tuning(self, row_tile=0, chunk=0, graphs=0):
        t = Tuning(int(row_tile), int(chunk), int(graphs), 0.0)
        _check(load().cpra_set_tuning(self.handle, ctypes.byref(t)), self.handle)

    def set_graphs(self, enable=True):
        """Replay whole episodes from captured HIP graphs (see cpra_set_graphs)."""
        _check(load().cpra_set_graphs(self.handle, int(bool(enable))), self.handle)

    def set_chunk(self, slots):
        """Chunk-major order inside episodes, `slots` per chunk; 0 turns it off (cpra_set_chunk)."""
        _check(load().cpra_set_chunk(self.handle, int(slots)), self.handle)

    def set_kernel_timing(self, enable=True):
        _check(load().cpra_set_kernel_timing(self.handle, int(bool(enable))), self.handle)

    def kernel_timing(self):
        """(col_ms, col_launches, row_ms, row_launches) since timing was enabled or last read."""
        cm, rm = ctypes.c_double(0), ctypes.c_double(0)
        cl, rl = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(load().cpra_kernel_timing(self.handle, ctypes.byref(cm), ctypes.byref(cl), ctypes.byref(rm),
                                         ctypes.byref(rl)), self.handle)
        return cm.value, cl.value, rm.value, rl.value

    @property
    def k(self):
        v = ctypes.c_int64(0)
        _check(load().cpra_iteration_count(self.handle, ctypes.byref(v)), self.handle)
        return v.value
