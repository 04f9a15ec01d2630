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
STRATEGIES = {"fused": 0, "multi_kernel": 1, "compact": 2, "per_cell": 3}
STRATEGY_NAMES = {v: k for k, v in STRATEGIES.items()}
TUNE_MAX = 16
OPT_STRATEGY, OPT_CHUNKS_PER_BLOCK, OPT_PAIRS_PER_LANE, OPT_WIDE_INDEX = 0, 1, 2, 3
LOSSES = {"mse": 0, "mae": 1}
PNET_INPUTS, PNET_PARAMS = 9, 337  # the probability network (include/compton.h)


class CSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Species(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("w", C.c_void_p), ("n", C.c_int64)]


class TuneResult(C.Structure):
    _fields_ = [("n", C.c_int32), ("best", C.c_int32), ("strategy", C.c_int32 * 16),
                ("chunks_per_block", C.c_int32 * 16), ("pairs_per_lane", C.c_int32 * 16), ("ms", C.c_float * 16)]


STAGES = ["prep", "pair", "compact", "collide", "finalize"]
STATS_INT = ["n_pairs", "n_collided", "n_clipped", "n_invalid", "n_fallback", "layout_error", "overflow"]
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
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so that both share one runtime (devices, streams, memory)
    import torch  # noqa: F401

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
    L.cs_compton_step_noalloc.argtypes = L.cs_compton_step.argtypes
    L.cs_compton_step_noalloc.restype = st
    L.cs_ntc_step.argtypes = [vp, C.c_int, Species, Species, vp, vp, i64, d, d, u64, u64, vp, vp]
    L.cs_ntc_step.restype = st
    L.cs_check_layout.argtypes = [vp, vp, i64, i64, vp]
    L.cs_check_layout.restype = st
    L.cs_pair_x.argtypes = [vp, C.c_int, Species, Species, i64, vp, vp]
    L.cs_pair_x.restype = st
    L.cs_sample_plain.argtypes = [vp, C.c_int, vp, vp, i64, vp, vp, vp]
    L.cs_sample_plain.restype = st
    L.cs_bin_particles.argtypes = [vp, C.c_int, vp, Species, Species, vp, i64, vp, vp]
    L.cs_bin_particles.restype = st
    L.cs_pnet_target.argtypes = [vp, vp, i64, vp, vp]
    L.cs_pnet_target.restype = st
    L.cs_pnet_forward.argtypes = [vp, vp, vp, i64, vp, vp]
    L.cs_pnet_forward.restype = st
    L.cs_pnet_grad.argtypes = [vp, vp, vp, vp, i64, C.c_int, vp, vp, vp]
    L.cs_pnet_grad.restype = st
    L.cs_pnet_adam.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, vp]
    L.cs_pnet_adam.restype = st
    L.cs_set_option.argtypes = [vp, C.c_int, i64]
    L.cs_set_option.restype = st
    L.cs_get_option.argtypes = [vp, C.c_int, C.POINTER(i64)]
    L.cs_get_option.restype = st
    L.cs_set_stage_timing.argtypes = [vp, C.c_int]
    L.cs_set_stage_timing.restype = st
    L.cs_stage_times.argtypes = [vp, C.POINTER(C.c_float), i32, C.POINTER(i32)]
    L.cs_stage_times.restype = st
    L.cs_autotune.argtypes = [vp, C.c_int, Species, Species, vp, vp, i64, d, d, u64, u64, C.c_int, vp, i32,
                              C.POINTER(TuneResult), vp]
    L.cs_autotune.restype = st
    L.cs_graph_create.argtypes = [vp, C.c_int, Species, Species, vp, vp, i64, d, d, u64, C.c_int, vp, vp, vp,
                                  C.POINTER(vp)]
    L.cs_graph_create.restype = st
    L.cs_ntc_graph_create.argtypes = [vp, C.c_int, Species, Species, vp, vp, i64, d, d, u64, i64, vp, vp,
                                      C.POINTER(vp)]
    L.cs_ntc_graph_create.restype = st
    L.cs_graph_set_step.argtypes = [vp, u64, vp]
    L.cs_graph_set_step.restype = st
    L.cs_graph_launch.argtypes = [vp, vp]
    L.cs_graph_launch.restype = st
    L.cs_graph_destroy.argtypes = [vp]
    L.cs_graph_destroy.restype = st
    _bind_mlp(L)
    _lib = L
    return L


def _bind_mlp(L):
    """Signatures of the network entry points."""
    vp, i64, i32, f = C.c_void_p, C.c_int64, C.c_int32, C.c_float
    st = C.c_int
    sigs = {
        "cs_mlp_create": ([vp, C.POINTER(i32), i32, vp, C.POINTER(vp)], st),
        "cs_mlp_destroy": ([vp], st),
        "cs_mlp_num_params": ([vp], i64),
        "cs_mlp_set_params": ([vp, vp, i64], st),
        "cs_mlp_get_params": ([vp, vp, i64], st),
        "cs_mlp_set_domain": ([vp, C.c_double, C.c_double], st),
        "cs_mlp_get_domain": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_double)], st),
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

    def step_noalloc(self, e, g, off_e, off_g, dt, density_norm, seed, step, sampler="plain", mlp=None, stats=None,
                     stream=None):
        """step through cs_compton_step_noalloc (no device allocation; the
        library's static scratch, shared by every call on the device)."""
        code = _dtype_code(e["x"])
        rc = lib().cs_compton_step_noalloc(self._h, code, _species(e), _species(g), _ptr(off_e), _ptr(off_g),
                                           off_e.numel() - 1, float(dt), float(density_norm), int(seed), int(step),
                                           SAMPLERS[sampler], None if mlp is None else mlp.handle, _ptr(stats),
                                           _stream(stream))
        self._check(rc)

    def ntc_step(self, e, g, off_e, off_g, dt, density_norm, seed, step, stats=None, stream=None):
        """One Compton step with no-time-counter candidate selection, in place
        on device tensors (the layout of step); queues the whole step, then
        waits for the device's candidate count."""
        code = _dtype_code(e["x"])
        rc = lib().cs_ntc_step(self._h, code, _species(e), _species(g), _ptr(off_e), _ptr(off_g),
                               off_e.numel() - 1, float(dt), float(density_norm), int(seed), int(step), _ptr(stats),
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

    def set_pairs_per_lane(self, n):
        self.set_option(OPT_PAIRS_PER_LANE, n)

    def set_wide_index(self, on):
        self.set_option(OPT_WIDE_INDEX, 1 if on else 0)

    def set_stage_timing(self, enable):
        self._check(lib().cs_set_stage_timing(self._h, 1 if enable else 0))

    def stage_times(self):
        """Milliseconds per stage of the last timed step (synchronous)."""
        buf = (C.c_float * 8)()
        n = C.c_int32()
        self._check(lib().cs_stage_times(self._h, buf, 8, C.byref(n)))
        return dict(zip(STAGES, [float(buf[i]) for i in range(n.value)]))

    def autotune(self, e, g, off_e, off_g, dt, density_norm, seed, step, sampler="plain", mlp=None, reps=5,
                 stream=None):
        """Time the candidate strategies on a private copy of the particles and
        keep the fastest; returns {"best": (strategy, chunks, pairs_per_lane),
        "candidates": [(strategy, chunks, pairs_per_lane, ms), ...]}."""
        res = TuneResult()
        rc = lib().cs_autotune(self._h, _dtype_code(e["x"]), _species(e), _species(g), _ptr(off_e), _ptr(off_g),
                               off_e.numel() - 1, float(dt), float(density_norm), int(seed), int(step),
                               SAMPLERS[sampler], None if mlp is None else mlp.handle, int(reps), C.byref(res),
                               _stream(stream))
        self._check(rc)
        cands = [(STRATEGY_NAMES[res.strategy[i]], int(res.chunks_per_block[i]), int(res.pairs_per_lane[i]),
                  float(res.ms[i])) for i in range(res.n)]
        return {"best": cands[res.best][:3], "candidates": cands}

    def graph(self, e, g, off_e, off_g, dt, density_norm, seed, sampler="plain", mlp=None, stats=None,
              stream=None):
        """Capture one step into a replayable graph (see Graph)."""
        return Graph(self, e, g, off_e, off_g, dt, density_norm, seed, sampler, mlp, stats, stream)

    def ntc_graph(self, e, g, off_e, off_g, dt, density_norm, seed, max_candidates, stats=None, stream=None):
        """Capture one NTC step (cs_ntc_graph_create) sized for max_candidates
        candidates per step; a replay that draws more changes nothing and sets
        stats' overflow word (see Graph)."""
        return Graph(self, e, g, off_e, off_g, dt, density_norm, seed, "plain", None, stats, stream,
                     ntc_max_candidates=max_candidates)

    def bin_particles(self, cell, species, n_cells, out=None, off=None, n_invalid=None, stream=None):
        """Group one species by cell (cs_bin_particles).  cell: int32 device
        tensor; species: dict of x, y, z, w device tensors.  Returns (out
        species dict, int64 offsets of n_cells + 1, int64 n_invalid tensor of
        one element); out from off[n_cells] on holds the particles with no
        valid cell, in input order."""
        import torch

        if out is None:
            out = {k: torch.empty_like(species[k]) for k in "xyzw"}
        dev = species["x"].device
        off = torch.empty(n_cells + 1, dtype=torch.int64, device=dev) if off is None else off
        n_invalid = torch.zeros(1, dtype=torch.int64, device=dev) if n_invalid is None else n_invalid
        rc = lib().cs_bin_particles(self._h, _dtype_code(species["x"]), _ptr(cell), _species(species),
                                    _species(out), _ptr(off), n_cells, _ptr(n_invalid), _stream(stream))
        self._check(rc)
        return out, off, n_invalid

    # -- the probability network (inputs: float32 device tensor [n, 9]) --
    def pnet_target(self, inputs, y_out=None, stream=None):
        import torch

        n = inputs.shape[0]
        y_out = torch.empty(n, dtype=torch.float32, device=inputs.device) if y_out is None else y_out
        self._check(lib().cs_pnet_target(self._h, _ptr(inputs), n, _ptr(y_out), _stream(stream)))
        return y_out

    def pnet_forward(self, params, inputs, y_out=None, stream=None):
        import torch

        n = inputs.shape[0]
        y_out = torch.empty(n, dtype=torch.float32, device=inputs.device) if y_out is None else y_out
        self._check(lib().cs_pnet_forward(self._h, _ptr(params), _ptr(inputs), n, _ptr(y_out), _stream(stream)))
        return y_out

    def pnet_grad(self, params, inputs, target, loss="mae", grad_out=None, loss_out=None, stream=None):
        import torch

        grad_out = torch.empty(PNET_PARAMS, dtype=torch.float32, device=params.device) if grad_out is None \
            else grad_out
        loss_out = torch.empty(1, dtype=torch.float32, device=params.device) if loss_out is None else loss_out
        self._check(lib().cs_pnet_grad(self._h, _ptr(params), _ptr(inputs), _ptr(target), inputs.shape[0],
                                       LOSSES[loss], _ptr(grad_out), _ptr(loss_out), _stream(stream)))
        return grad_out, loss_out

    def pnet_adam(self, params, grad, m, v, t, lr=1e-3, stream=None):
        self._check(lib().cs_pnet_adam(self._h, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), t, lr,
                                       _stream(stream)))

    def pair_x(self, e, g, n=None, x_out=None, stream=None):
        """Rest-frame photon energies (float64 device tensor) of the pairs
        (electron i, photon i), i < n (default: the smaller species count)."""
        import torch

        n = min(e["x"].numel(), g["x"].numel()) if n is None else int(n)
        x_out = torch.empty(n, dtype=torch.float64, device=e["x"].device) if x_out is None else x_out
        rc = lib().cs_pair_x(self._h, _dtype_code(e["x"]), _species(e), _species(g), n, _ptr(x_out),
                             _stream(stream))
        self._check(rc)
        return x_out

    def sample_plain(self, x, u, mu_out=None, ratio_out=None, stream=None):
        import torch

        mu_out = torch.empty_like(x) if mu_out is None else mu_out
        ratio_out = torch.empty_like(x) if ratio_out is None else ratio_out
        rc = lib().cs_sample_plain(self._h, _dtype_code(x), _ptr(x), _ptr(u), x.numel(), _ptr(mu_out),
                                   _ptr(ratio_out), _stream(stream))
        self._check(rc)
        return mu_out, ratio_out


class Graph:
    """One captured step: replays take the step index from a device counter
    (set_step) that each replay advances.  The tensors given at capture must
    stay alive (and in place) while the graph is used; the stream must not be
    the legacy default stream."""

    def __init__(self, ctx, e, g, off_e, off_g, dt, density_norm, seed, sampler, mlp, stats, stream,
                 ntc_max_candidates=None):
        import torch

        self.ctx = ctx
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self._keep = (e, g, off_e, off_g, stats, mlp)
        self._h = C.c_void_p()
        if ntc_max_candidates is None:
            rc = lib().cs_graph_create(ctx.handle, _dtype_code(e["x"]), _species(e), _species(g), _ptr(off_e),
                                       _ptr(off_g), off_e.numel() - 1, float(dt), float(density_norm), int(seed),
                                       SAMPLERS[sampler], None if mlp is None else mlp.handle, _ptr(stats),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        else:
            rc = lib().cs_ntc_graph_create(ctx.handle, _dtype_code(e["x"]), _species(e), _species(g), _ptr(off_e),
                                           _ptr(off_g), off_e.numel() - 1, float(dt), float(density_norm),
                                           int(seed), int(ntc_max_candidates), _ptr(stats),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        ctx._check(rc)

    def set_step(self, step):
        self.ctx._check(lib().cs_graph_set_step(self._h, int(step), C.c_void_p(self.stream.cuda_stream)))

    def launch(self):
        self.ctx._check(lib().cs_graph_launch(self._h, C.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if self._h:
            lib().cs_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


WIDTHS = (2, 64, 64, 64, 64, 2)
X_MIN, X_MAX = 1e-4, 1e2  # the default x range of a network


class MLP:
    """The sampler network on one device: FP32 parameters, Adam state and the
    BF16 / FP8 copies the MFMA kernels read.  Parameters cross the boundary as
    a flat float32 vector (per layer W[n_out, n_in] row-major, then b)."""

    def __init__(self, ctx, params=None, _handle=None):
        self.ctx = ctx
        if _handle is not None:
            self._h = _handle
            return
        self._h = C.c_void_p()
        w = (C.c_int32 * len(WIDTHS))(*WIDTHS)
        host = None
        if params is not None:
            host = np.ascontiguousarray(params, dtype=np.float32)
        rc = lib().cs_mlp_create(ctx.handle, w, len(WIDTHS),
                                 None if host is None else host.ctypes.data_as(C.c_void_p), C.byref(self._h))
        ctx._check(rc)

    @classmethod
    def load(cls, ctx, path):
        h = C.c_void_p()
        ctx._check(lib().cs_mlp_load(ctx.handle, os.fsencode(path), C.byref(h)))
        return cls(ctx, _handle=h)

    @property
    def handle(self):
        return self._h

    @property
    def n_params(self):
        return int(lib().cs_mlp_num_params(self._h))

    def close(self):
        if self._h:
            lib().cs_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc, what):
        if rc != CS_OK:
            raise CSError(rc, what)

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        self._rc(lib().cs_mlp_get_params(self._h, out.ctypes.data_as(C.c_void_p), out.size), "cs_mlp_get_params")
        return out

    def set_params(self, params):
        host = np.ascontiguousarray(params, dtype=np.float32)
        self._rc(lib().cs_mlp_set_params(self._h, host.ctypes.data_as(C.c_void_p), host.size), "cs_mlp_set_params")

    def set_domain(self, x_min, x_max):
        """The x range the network answers for (its first feature maps log10 x
        from this range onto [-1, 1]; outside it the plain sampler answers)."""
        rc = lib().cs_mlp_set_domain(self._h, float(x_min), float(x_max))
        self._rc(rc, f"cs_mlp_set_domain({x_min}, {x_max})")

    @property
    def domain(self):
        lo, hi = C.c_double(), C.c_double()
        self._rc(lib().cs_mlp_get_domain(self._h, C.byref(lo), C.byref(hi)), "cs_mlp_get_domain")
        return lo.value, hi.value

    def save(self, path):
        self._rc(lib().cs_mlp_save(self._h, os.fsencode(path)), f"cs_mlp_save({path})")

    def quantize(self, precision, calib_x=None, calib_u=None, stream=None):
        n = 0 if calib_x is None else calib_x.numel()
        self.ctx._check(lib().cs_mlp_quantize(self.ctx.handle, self._h, SAMPLERS[precision], _ptr(calib_x),
                                              _ptr(calib_u), n, _stream(stream)))

    def forward(self, x, u, precision="mlp_f32", y_out=None, stream=None):
        """Raw outputs y[n, 2] (float32 device tensor)."""
        import torch

        y_out = torch.empty((x.numel(), 2), dtype=torch.float32, device=x.device) if y_out is None else y_out
        self.ctx._check(lib().cs_mlp_forward(self.ctx.handle, self._h, SAMPLERS[precision], _ptr(x), _ptr(u),
                                             x.numel(), _ptr(y_out), _stream(stream)))
        return y_out

    def sample(self, x, u, precision="mlp_f32", stream=None):
        """(mu, ratio, fallback mask) for x, u (float32 device tensors)."""
        import torch

        mu = torch.empty_like(x)
        r = torch.empty_like(x)
        mask = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
        self.ctx._check(lib().cs_mlp_sample(self.ctx.handle, self._h, SAMPLERS[precision], _ptr(x), _ptr(u),
                                            x.numel(), _ptr(mu), _ptr(r), _ptr(mask), _stream(stream)))
        return mu, r, mask

    def grad(self, x, u, mu_t, r_t, loss="mse", stream=None):
        """(loss, gradient) as device tensors (shape [], [n_params])."""
        import torch

        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        l = torch.empty((), dtype=torch.float32, device=x.device)
        self.ctx._check(lib().cs_mlp_grad(self.ctx.handle, self._h, _ptr(x), _ptr(u), _ptr(mu_t), _ptr(r_t),
                                          x.numel(), LOSSES[loss], _ptr(g), _ptr(l), _stream(stream)))
        return l, g

    def adam_step(self, grad, lr=1e-3, stream=None):
        self.ctx._check(lib().cs_mlp_adam_step(self.ctx.handle, self._h, _ptr(grad), float(lr), _stream(stream)))

    def train_step(self, x, u, mu_t, r_t, lr=1e-3, loss="mse", loss_out=None, stream=None):
        """One optimiser step on the batch; the loss (before the update) is
        written to loss_out (a float32 device scalar) when given."""
        self.ctx._check(lib().cs_mlp_train_step(self.ctx.handle, self._h, _ptr(x), _ptr(u), _ptr(mu_t), _ptr(r_t),
                                                x.numel(), float(lr), LOSSES[loss], _ptr(loss_out),
                                                _stream(stream)))


def to_device(p, device="cuda:0"):
    """Host Plasma (numpy) -> dict of device tensors (e, g, off_e, off_g)."""
    import torch

    e = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in p.e.items()}
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in p.g.items()}
    return e, g, torch.from_numpy(p.off_e).to(device), torch.from_numpy(p.off_g).to(device)


def to_host(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}
