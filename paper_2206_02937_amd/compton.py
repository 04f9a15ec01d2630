"""ctypes binding of libcompton.so (declared in include/compton.h).

Argument marshalling only: torch tensors provide device memory, the current
torch stream provides the hipStream_t, and every step of the computation runs
in the library's HIP kernels.  There is no fallback: if the library is not
built, or a call fails, an exception is raised.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcompton.so")

CS_OK, CS_ERR_INVALID_ARG, CS_ERR_LAYOUT, CS_ERR_UNSUPPORTED, CS_ERR_HIP, CS_ERR_IO, CS_ERR_NOT_READY = range(7)
STATUS_NAMES = {0: "CS_OK", 1: "CS_ERR_INVALID_ARG", 2: "CS_ERR_LAYOUT", 3: "CS_ERR_UNSUPPORTED",
                4: "CS_ERR_HIP", 5: "CS_ERR_IO", 6: "CS_ERR_NOT_READY"}
CS_F32, CS_F64 = 0, 1
SAMPLERS = {"plain": 0, "mlp_f32": 1, "mlp_bf16": 2, "mlp_fp8": 3}
STRATEGIES = {"fused": 0, "multi_kernel": 1, "compact": 2}
OPT_STRATEGY, OPT_CHUNKS_PER_BLOCK = 0, 1
LOSSES = {"mse": 0, "mae": 1}


class CSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Species(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("w", C.c_void_p), ("n", C.c_int64)]


STAGES = ["prep", "pair", "compact", "collide", "finalize"]
STATS_INT = ["n_pairs", "n_collided", "n_clipped", "n_invalid", "n_fallback", "layout_error"]
STATS_DBL = ["sum_prob", "energy_before", "energy_after"]
STATS_BYTES = 128

_lib = None


def lib():
    """Load libcompton.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_02937_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, u64, d, i32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_double, C.c_int32
    st = C.c_int
    L.cs_create.argtypes = [C.POINTER(vp), C.c_int]
    L.cs_create.restype = st
    L.cs_destroy.argtypes = [vp]
    L.cs_destroy.restype = st
    L.cs_last_error.argtypes = [vp]
    L.cs_last_error.restype = C.c_char_p
    L.cs_sync.argtypes = [vp, vp]
    L.cs_sync.restype = st
    L.cs_compton_step.argtypes = [vp, C.c_int, Species, Species, vp, vp, i64, d, d, u64, u64, C.c_int, vp, vp, vp]
    L.cs_compton_step.restype = st
    L.cs_check_layout.argtypes = [vp, vp, i64, i64, vp]
    L.cs_check_layout.restype = st
    L.cs_sample_plain.argtypes = [vp, C.c_int, vp, vp, i64, vp, vp, vp]
    L.cs_sample_plain.restype = st
    L.cs_set_option.argtypes = [vp, C.c_int, i64]
    L.cs_set_option.restype = st
    L.cs_get_option.argtypes = [vp, C.c_int, C.POINTER(i64)]
    L.cs_get_option.restype = st
    L.cs_set_stage_timing.argtypes = [vp, C.c_int]
    L.cs_set_stage_timing.restype = st
    L.cs_stage_times.argtypes = [vp, C.POINTER(C.c_float), i32, C.POINTER(i32)]
    L.cs_stage_times.restype = st
    _optional(L)
    _lib = L
    return L


def _optional(L):
    """Bind the network entry points when the library exports them."""
    vp, i64, u64, i32, f = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.c_float
    st = C.c_int
    sigs = {
        "cs_mlp_create": ([vp, C.POINTER(i32), i32, vp, C.POINTER(vp)], st),
        "cs_mlp_destroy": ([vp], st),
        "cs_mlp_num_params": ([vp], i64),
        "cs_mlp_set_params": ([vp, vp, i64], st),
        "cs_mlp_get_params": ([vp, vp, i64], st),
        "cs_mlp_save": ([vp, C.c_char_p], st),
        "cs_mlp_load": ([vp, C.c_char_p, C.POINTER(vp)], st),
        "cs_mlp_quantize": ([vp, vp, C.c_int, vp, vp, i64, vp], st),
        "cs_mlp_sample": ([vp, vp, C.c_int, vp, vp, i64, vp, vp, vp, vp], st),
        "cs_mlp_forward": ([vp, vp, C.c_int, vp, vp, i64, vp, vp], st),
        "cs_mlp_grad": ([vp, vp, vp, vp, vp, vp, i64, C.c_int, vp, vp, vp], st),
        "cs_mlp_adam_step": ([vp, vp, vp, f, vp], st),
        "cs_mlp_train_step": ([vp, vp, vp, vp, vp, vp, i64, f, C.c_int, vp, vp], st),
    }
    for name, (args, res) in sigs.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _species(d):
    n = d["x"].numel()
    return Species(d["x"].data_ptr(), d["y"].data_ptr(), d["z"].data_ptr(), d["w"].data_ptr(), n)


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return CS_F64
    if t.dtype == torch.float32:
        return CS_F32
    raise CSError(CS_ERR_INVALID_ARG, f"unsupported dtype {t.dtype}")


def decode_stats(t):
    """cs_stats (a 128-byte device or host tensor) -> dict."""
    raw = t.detach().cpu().numpy().view(np.uint8).tobytes()
    ints = np.frombuffer(raw[:64], dtype=np.int64)
    dbls = np.frombuffer(raw[64:], dtype=np.float64)
    out = {k: int(ints[i]) for i, k in enumerate(STATS_INT)}
    out.update({k: float(dbls[i]) for i, k in enumerate(STATS_DBL)})
    return out


class Context:
    """A library context on one device (workspace, error text)."""

    def __init__(self, device=0):
        self._h = C.c_void_p()
        rc = lib().cs_create(C.byref(self._h), int(device))
        if rc != CS_OK:
            raise CSError(rc, lib().cs_last_error(None).decode())
        self.device = device

    @property
    def handle(self):
        return self._h

    def _check(self, rc):
        if rc != CS_OK:
            raise CSError(rc, lib().cs_last_error(self._h).decode())

    def close(self):
        if self._h:
            lib().cs_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None):
        self._check(lib().cs_sync(self._h, _stream(stream)))

    def stats_buffer(self):
        import torch

        return torch.zeros(STATS_BYTES // 8, dtype=torch.int64, device=f"cuda:{self.device}")

    def step(self, e, g, off_e, off_g, dt, density_norm, seed, step, sampler="plain", mlp=None, stats=None,
             stream=None):
        """One Compton step in place on device tensors (dicts with x, y, z, w)."""
        code = _dtype_code(e["x"])
        rc = lib().cs_compton_step(self._h, code, _species(e), _species(g), _ptr(off_e), _ptr(off_g),
                                   off_e.numel() - 1, float(dt), float(density_norm), int(seed), int(step),
                                   SAMPLERS[sampler], None if mlp is None else mlp.handle, _ptr(stats),
                                   _stream(stream))
        self._check(rc)

    def check_layout(self, off, n, stream=None):
        rc = lib().cs_check_layout(self._h, _ptr(off), off.numel() - 1, int(n), _stream(stream))
        if rc == CS_ERR_LAYOUT:
            return False
        self._check(rc)
        return True

    def set_option(self, opt, value):
        self._check(lib().cs_set_option(self._h, int(opt), int(value)))

    def get_option(self, opt):
        v = C.c_int64()
        self._check(lib().cs_get_option(self._h, int(opt), C.byref(v)))
        return v.value

    def set_strategy(self, name):
        self.set_option(OPT_STRATEGY, STRATEGIES[name])

    def set_chunks_per_block(self, g):
        self.set_option(OPT_CHUNKS_PER_BLOCK, g)

    def set_stage_timing(self, enable):
        self._check(lib().cs_set_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """Milliseconds per stage of the last timed step (synchronous)."""
        buf = (C.c_float * 8)()
        n = C.c_int32()
        self._check(lib().cs_stage_times(self._h, buf, 8, C.byref(n)))
        return dict(zip(STAGES, [float(buf[i]) for i in range(n.value)]))

    def sample_plain(self, x, u, mu_out=None, ratio_out=None, stream=None):
        import torch

        mu_out = torch.empty_like(x) if mu_out is None else mu_out
        ratio_out = torch.empty_like(x) if ratio_out is None else ratio_out
        rc = lib().cs_sample_plain(self._h, _dtype_code(x), _ptr(x), _ptr(u), x.numel(), _ptr(mu_out),
                                   _ptr(ratio_out), _stream(stream))
        self._check(rc)
        return mu_out, ratio_out


def to_device(p, device="cuda:0"):
    """Host Plasma (numpy) -> dict of device tensors (e, g, off_e, off_g)."""
    import torch

    e = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in p.e.items()}
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in p.g.items()}
    return e, g, torch.from_numpy(p.off_e).to(device), torch.from_numpy(p.off_g).to(device)


def to_host(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}
