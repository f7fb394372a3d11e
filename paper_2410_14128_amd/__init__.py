"""Ray intersection through hybrid voxel formats on MI355X: Python binding of libhvf.so.

Argument marshalling only. Every step of building and tracing runs in the native
library (host C++ builder, HIP kernels); there is no Python or CPU fallback, and
importing this module without a built libhvf.so raises.

PyTorch supplies device memory and streams: ``Volume.trace`` takes CUDA (HIP) tensors
of rays (float32 [n, 8]: ox, oy, oz, tmin, dx, dy, dz, tmax) and hits (int32 [n, 4]:
x, y, z and the float32 bits of t).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libhvf.so")

HVF_MAX_LEVELS = 8
HVF_MAX_DEPTH = 16

STATUS = {0: "HVF_OK", 1: "HVF_E_SPEC", 2: "HVF_E_INPUT", 3: "HVF_E_OVERFLOW", 4: "HVF_E_NOMEM",
          5: "HVF_E_DEVICE", 6: "HVF_E_UNSUPPORTED", 7: "HVF_E_STATE"}


class HvfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class hvf_info(ctypes.Structure):
    _fields_ = [
        ("num_levels", ctypes.c_int32),
        ("kinds", ctypes.c_char * HVF_MAX_LEVELS),
        ("level_exp", (ctypes.c_int32 * 3) * HVF_MAX_LEVELS),
        ("extent_log2", ctypes.c_int32 * 3),
        ("whole_level_dedup", ctypes.c_int32),
        ("num_depths", ctypes.c_int32),
        ("num_words", ctypes.c_uint64),
        ("level_nodes", ctypes.c_uint64 * HVF_MAX_LEVELS),
        ("depth_nodes", ctypes.c_uint64 * HVF_MAX_DEPTH),
        ("depth_offset", ctypes.c_uint64 * HVF_MAX_DEPTH),
        ("num_voxels", ctypes.c_uint64),
        ("level_maxdist", ctypes.c_int32 * HVF_MAX_LEVELS),
        ("kernel_family", ctypes.c_uint32), ("paper_layout", ctypes.c_int32), ("depth_buffers", ctypes.c_int32),
    ]


class hvf_schedule(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("refill", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("sort", ctypes.c_int32), ("sort_bits", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("stack_depth", ctypes.c_int32), ("lds_depths", ctypes.c_int32), ("split", ctypes.c_int32),
                ("split_budget", ctypes.c_int32), ("split_rounds", ctypes.c_int32), ("steal", ctypes.c_int32),
                ("steal_len", ctypes.c_int32), ("steal_idle", ctypes.c_int32), ("interleave", ctypes.c_int32),
                ("rays_per_wave", ctypes.c_int32)]


def schedule(persistent: int = 0, refill: int = 16, inner: int = 8, sort: int = 0, sort_bits: int = 4,
             blocks_per_cu: int = 0, stack_depth: int = 0, lds_depths: int = 0, split: int = 0,
             split_budget: int = 0, split_rounds: int = 0, steal: int = 0, steal_len: int = 0,
             steal_idle: int = 1, interleave: int = 0, rays_per_wave: int = 0) -> hvf_schedule:
    """A device schedule for a trace (results never depend on it)."""
    return hvf_schedule(persistent, refill, inner, sort, sort_bits, blocks_per_cu, stack_depth, lds_depths, split,
                        split_budget, split_rounds, steal, steal_len, steal_idle, interleave, rays_per_wave)


def kernel_names(info: dict, sched: dict) -> list:
    """Demangled-name stems of the kernels a volume launches under a schedule, in order."""
    fam = info["kernel_family"]
    if sched.get("sort"):
        return ["trace_indexed_kernel"]
    if sched.get("split"):
        resume = [f"trace_resume_kernel<{fam}u>"] if sched.get("split_rounds") else []
        return [f"trace_budget_kernel<{fam}u>"] + resume + [f"trace_split_kernel<{fam}u>"]
    if sched.get("steal"):
        return [f"trace_steal_kernel<{fam}u>"]
    kind = "trace_persistent_kernel" if sched.get("persistent") else "trace_kernel"
    return [f"{kind}<{fam}u>"]


def kernel_name(info: dict, sched: dict) -> str:
    """The kernel names of kernel_names joined by ' + ' (one trace call)."""
    return " + ".join(kernel_names(info, sched))


def schedule_dict(s: hvf_schedule) -> dict:
    return {"persistent": s.persistent, "refill": s.refill, "inner": s.inner, "sort": s.sort, "sort_bits": s.sort_bits,
            "blocks_per_cu": s.blocks_per_cu, "stack_depth": s.stack_depth, "lds_depths": s.lds_depths,
            "split": s.split, "split_budget": s.split_budget, "split_rounds": s.split_rounds, "steal": s.steal,
            "steal_len": s.steal_len, "steal_idle": s.steal_idle, "interleave": s.interleave,
            "rays_per_wave": s.rays_per_wave}


class hvf_batch_opts(ctypes.Structure):
    _fields_ = [("refill", ctypes.c_int32), ("inner", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


def batch_opts(refill: int = 16, inner: int = 8, blocks_per_cu: int = 0, use_graph: int = 1) -> hvf_batch_opts:
    return hvf_batch_opts(refill, inner, blocks_per_cu, use_graph)


class hvf_serve_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("rays", ctypes.c_uint64),
                ("span_ms", ctypes.c_double), ("mrays_s", ctypes.c_double), ("steps", ctypes.c_uint64),
                ("admission_waits", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("max_step_requests", ctypes.c_uint64)]


_lib = None


NOALLOC_MAX_RAYS = 1 << 21  # HVF_NOALLOC_MAX_RAYS


def lib():
    """Load libhvf.so (built by ``paper_2410_14128_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise ImportError(f"{SO_PATH} is not built; run `python -m paper_2410_14128_amd.build` "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(SO_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        L.hvf_build.restype = i32
        L.hvf_build.argtypes = [ctypes.c_char_p, vp, sz, ctypes.POINTER(vp)]
        L.hvf_build_device.restype = i32
        L.hvf_build_device.argtypes = [ctypes.c_char_p, vp, sz, vp, ctypes.POINTER(vp)]
        L.hvf_upload.restype = i32
        L.hvf_upload.argtypes = [vp, vp]
        L.hvf_trace.restype = i32
        L.hvf_trace.argtypes = [vp, vp, sz, vp, vp]
        L.hvf_trace_sched.restype = i32
        L.hvf_trace_sched.argtypes = [vp, vp, sz, vp, ctypes.POINTER(hvf_schedule), vp]
        L.hvf_trace_split_noalloc.restype = i32
        L.hvf_trace_split_noalloc.argtypes = [vp, vp, sz, vp, ctypes.POINTER(hvf_schedule), vp]
        L.hvf_get_schedule.restype = i32
        L.hvf_get_schedule.argtypes = [vp, ctypes.POINTER(hvf_schedule)]
        L.hvf_set_schedule.restype = i32
        L.hvf_set_schedule.argtypes = [vp, ctypes.POINTER(hvf_schedule)]
        L.hvf_autotune.restype = i32
        L.hvf_autotune.argtypes = [vp, vp, sz, vp, ctypes.POINTER(hvf_schedule), vp]
        L.hvf_batch_create.restype = i32
        L.hvf_batch_create.argtypes = [vp, vp, vp, vp, sz, ctypes.POINTER(hvf_batch_opts), ctypes.POINTER(vp)]
        L.hvf_batch_run.restype = i32
        L.hvf_batch_run.argtypes = [vp, vp]
        L.hvf_batch_autotune.restype = i32
        L.hvf_batch_autotune.argtypes = [vp, vp, ctypes.POINTER(hvf_batch_opts)]
        L.hvf_batch_free.restype = None
        L.hvf_batch_free.argtypes = [vp]
        L.hvf_server_create.restype = i32
        L.hvf_server_create.argtypes = [sz, i32, i32, ctypes.POINTER(hvf_batch_opts), ctypes.POINTER(vp)]
        L.hvf_server_add_volume.restype = i32
        L.hvf_server_add_volume.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.hvf_server_submit.restype = i32
        L.hvf_server_submit.argtypes = [vp, i32, vp, sz, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.hvf_server_poll.restype = i32
        L.hvf_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        L.hvf_server_wait.restype = i32
        L.hvf_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.hvf_server_result.restype = i32
        L.hvf_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
        L.hvf_server_release.restype = i32
        L.hvf_server_release.argtypes = [vp, ctypes.c_uint64]
        L.hvf_server_drain.restype = i32
        L.hvf_server_drain.argtypes = [vp]
        L.hvf_server_fail_steps.restype = i32
        L.hvf_server_fail_steps.argtypes = [vp, ctypes.c_int]
        L.hvf_server_stats.restype = i32
        L.hvf_server_stats.argtypes = [vp, ctypes.POINTER(hvf_serve_stats)]
        L.hvf_server_destroy.restype = None
        L.hvf_server_destroy.argtypes = [vp]
        L.hvf_trace_count.restype = i32
        L.hvf_trace_count.argtypes = [vp, vp, sz, vp, vp, ctypes.c_uint32, vp, vp, vp]
        L.hvf_trace_host.restype = i32
        L.hvf_trace_host.argtypes = [vp, vp, sz, vp]
        L.hvf_info_get.restype = i32
        L.hvf_info_get.argtypes = [vp, ctypes.POINTER(hvf_info)]
        L.hvf_words.restype = i32
        L.hvf_words.argtypes = [vp, vp, sz, ctypes.POINTER(sz)]
        L.hvf_save.restype = i32
        L.hvf_save.argtypes = [vp, ctypes.c_char_p]
        L.hvf_load.restype = i32
        L.hvf_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        L.hvf_free.restype = None
        L.hvf_free.argtypes = [vp]
        L.hvf_status_string.restype = ctypes.c_char_p
        L.hvf_status_string.argtypes = [i32]
        L.hvf_last_error.restype = ctypes.c_char_p
        L.hvf_last_error.argtypes = []
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise HvfError(st, lib().hvf_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Volume:
    """A built hybrid format (host word buffer; device copy made on first trace)."""

    def __init__(self, spec: str, codes: np.ndarray | None = None, *, _handle=None):
        if _handle is not None:
            self._h = _handle
        else:
            c = np.ascontiguousarray(codes if codes is not None else np.zeros(0), dtype=np.uint64)
            h = ctypes.c_void_p()
            _check(lib().hvf_build(spec.encode(), c.ctypes.data if len(c) else None, len(c), ctypes.byref(h)))
            self._h = h.value
        self.spec = spec

    @classmethod
    def from_device(cls, spec: str, codes, stream=None) -> "Volume":
        """Build on the device from a uint64 (or int64) CUDA tensor of ascending Morton codes."""
        import torch
        if not isinstance(codes, torch.Tensor) or not codes.is_cuda:
            raise TypeError("codes must be a device tensor")
        if codes.dtype not in (torch.int64, torch.uint64) or codes.dim() != 1:
            raise TypeError("codes must be a 1-D 64-bit integer tensor")
        c = codes.contiguous()
        h = ctypes.c_void_p()
        n = c.numel()
        _check(lib().hvf_build_device(spec.encode(), c.data_ptr() if n else None, n, _stream_ptr(stream),
                                      ctypes.byref(h)))
        return cls(spec, _handle=h.value)

    @classmethod
    def load(cls, path: str) -> "Volume":
        h = ctypes.c_void_p()
        _check(lib().hvf_load(path.encode(), ctypes.byref(h)))
        v = cls("", _handle=h.value)
        return v

    def save(self, path: str):
        _check(lib().hvf_save(self._h, path.encode()))

    def close(self):
        if getattr(self, "_h", None):
            lib().hvf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        return self._h

    def info(self) -> dict:
        I = hvf_info()
        _check(lib().hvf_info_get(self._h, ctypes.byref(I)))
        n = I.num_levels
        nd = I.num_depths
        return {
            "num_levels": n,
            "kinds": I.kinds[:n].decode(),
            "level_exp": [tuple(I.level_exp[k]) for k in range(n)],
            "extent_log2": tuple(I.extent_log2),
            "whole_level_dedup": bool(I.whole_level_dedup),
            "num_depths": nd,
            "num_words": int(I.num_words),
            "bytes": int(I.num_words) * 4,
            "level_nodes": [int(I.level_nodes[k]) for k in range(n)],
            "depth_nodes": [int(I.depth_nodes[d]) for d in range(nd)],
            "depth_offset": [int(I.depth_offset[d]) for d in range(nd)],
            "num_voxels": int(I.num_voxels),
            "level_maxdist": [int(I.level_maxdist[k]) for k in range(n)],
            "kernel_family": int(I.kernel_family),
            "paper_layout": bool(I.paper_layout),
            "depth_buffers": bool(I.depth_buffers),
        }

    def words(self) -> np.ndarray:
        n = ctypes.c_size_t()
        _check(lib().hvf_words(self._h, None, 0, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.uint32)
        _check(lib().hvf_words(self._h, out.ctypes.data, n.value, ctypes.byref(n)))
        return out

    def upload(self, stream=None):
        _check(lib().hvf_upload(self._h, _stream_ptr(stream)))

    def trace(self, rays, hits=None, stream=None, sched: hvf_schedule | None = None):
        """Trace device rays (torch float32 [n, 8] on the GPU) into hits (int32 [n, 4]).

        Asynchronous on ``stream`` (default: torch's current stream). ``sched`` overrides
        the volume's schedule for this call. Returns ``hits``.
        """
        import torch
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.shape[-1] == 8 and rays.is_contiguous()
        n = rays.shape[0]
        if hits is None:
            hits = torch.empty((n, 4), dtype=torch.int32, device=rays.device)
        assert hits.is_cuda and hits.dtype == torch.int32 and hits.shape == (n, 4) and hits.is_contiguous()
        if sched is None:
            _check(lib().hvf_trace(self._h, rays.data_ptr(), n, hits.data_ptr(), _stream_ptr(stream)))
        else:
            _check(lib().hvf_trace_sched(self._h, rays.data_ptr(), n, hits.data_ptr(), ctypes.byref(sched),
                                         _stream_ptr(stream)))
        return hits

    def trace_split_noalloc(self, rays, hits, sched: hvf_schedule, stream=None):
        """hvf_trace_split_noalloc: a split-schedule trace whose scratch is the library's fixed
        device array (no allocation; the volume must be uploaded). Returns ``hits``."""
        import torch
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.shape[-1] == 8 and rays.is_contiguous()
        n = rays.shape[0]
        assert hits.is_cuda and hits.dtype == torch.int32 and hits.shape == (n, 4) and hits.is_contiguous()
        _check(lib().hvf_trace_split_noalloc(self._h, rays.data_ptr(), n, hits.data_ptr(), ctypes.byref(sched),
                                             _stream_ptr(stream)))
        return hits

    def autotune(self, sample_rays, stream=None) -> hvf_schedule:
        """Pick the fastest schedule on a device ray sample; it becomes this volume's."""
        import torch
        assert sample_rays.is_cuda and sample_rays.dtype == torch.float32 and sample_rays.is_contiguous()
        n = sample_rays.shape[0]
        scratch = torch.empty((n, 4), dtype=torch.int32, device=sample_rays.device)
        out = hvf_schedule()
        _check(lib().hvf_autotune(self._h, sample_rays.data_ptr(), n, scratch.data_ptr(), ctypes.byref(out),
                                  _stream_ptr(stream)))
        return out

    def get_schedule(self) -> hvf_schedule:
        s = hvf_schedule()
        _check(lib().hvf_get_schedule(self._h, ctypes.byref(s)))
        return s

    def set_schedule(self, sched: hvf_schedule):
        _check(lib().hvf_set_schedule(self._h, ctypes.byref(sched)))

    def trace_count(self, rays, cap: int = 4096, stream=None, steps: bool = False):
        """Counting variant: returns (hits, log int32 [n, cap] of word indices, count [n]),
        plus per-ray traversal step counts when ``steps``."""
        import torch
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.shape[-1] == 8 and rays.is_contiguous()
        n = rays.shape[0]
        hits = torch.empty((n, 4), dtype=torch.int32, device=rays.device)
        log = torch.empty((n, cap), dtype=torch.int32, device=rays.device)
        cnt = torch.empty((n,), dtype=torch.int32, device=rays.device)
        st = torch.empty((n,), dtype=torch.int32, device=rays.device) if steps else None
        _check(lib().hvf_trace_count(self._h, rays.data_ptr(), n, hits.data_ptr(), log.data_ptr(), cap,
                                     cnt.data_ptr(), st.data_ptr() if steps else None, _stream_ptr(stream)))
        return (hits, log, cnt, st) if steps else (hits, log, cnt)

    def trace_host(self, rays: np.ndarray) -> np.ndarray:
        """Synchronous host-array form: float32 [n, 8] in, int32 [n, 4] out."""
        r = np.ascontiguousarray(rays, dtype=np.float32)
        assert r.ndim == 2 and r.shape[1] == 8
        out = np.empty((len(r), 4), dtype=np.int32)
        _check(lib().hvf_trace_host(self._h, r.ctypes.data, len(r), out.ctypes.data))
        return out


class Batch:
    """Many volumes and ray batches traced in one persistent, graph-captured launch.

    ``vols``: Volume objects; ``rays``: device float32 [n_i, 8] tensors; ``hits``: device
    int32 [n_i, 4] tensors (allocated if None). The buffers are bound at creation.
    """

    def __init__(self, vols, rays, hits=None, opts: hvf_batch_opts | None = None):
        import torch
        m = len(vols)
        assert m == len(rays) and m >= 1
        if hits is None:
            hits = [torch.empty((r.shape[0], 4), dtype=torch.int32, device=r.device) for r in rays]
        for r, h in zip(rays, hits):
            assert r.is_cuda and r.dtype == torch.float32 and r.is_contiguous() and r.shape[-1] == 8
            assert h.is_cuda and h.dtype == torch.int32 and h.is_contiguous() and h.shape == (r.shape[0], 4)
        self.vols, self.rays, self.hits = list(vols), list(rays), list(hits)
        VP = ctypes.c_void_p * m
        SZ = ctypes.c_size_t * m
        hv = VP(*[v.handle for v in vols])
        rv = VP(*[r.data_ptr() for r in rays])
        nv = SZ(*[r.shape[0] for r in rays])
        ov = VP(*[h.data_ptr() for h in hits])
        out = ctypes.c_void_p()
        _check(lib().hvf_batch_create(ctypes.cast(hv, ctypes.c_void_p), ctypes.cast(rv, ctypes.c_void_p),
                                      ctypes.cast(nv, ctypes.c_void_p), ctypes.cast(ov, ctypes.c_void_p), m,
                                      ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
        self._h = out.value

    def run(self, stream=None):
        _check(lib().hvf_batch_run(self._h, _stream_ptr(stream)))
        return self.hits

    def autotune(self, stream=None) -> hvf_batch_opts:
        o = hvf_batch_opts()
        _check(lib().hvf_batch_autotune(self._h, _stream_ptr(stream), ctypes.byref(o)))
        return o

    def close(self):
        if getattr(self, "_h", None):
            lib().hvf_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Resident volumes, memory-gated admission, continuous batching (see include/hvf.h)."""

    def __init__(self, mem_budget_bytes: int, max_slots: int = 64, max_steps: int = 3,
                 opts: hvf_batch_opts | None = None):
        out = ctypes.c_void_p()
        _check(lib().hvf_server_create(mem_budget_bytes, max_slots, max_steps,
                                       ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
        self._h = out.value
        self._keep = {}  # request id -> (rays, hits) host arrays kept alive until completion

    def add_volume(self, vol: "Volume") -> int:
        vid = ctypes.c_int()
        _check(lib().hvf_server_add_volume(self._h, vol.handle, ctypes.byref(vid)))
        return vid.value

    def submit(self, vol_id: int, rays: np.ndarray, hits: np.ndarray | None = None, hold: bool = False) -> int:
        """Queue a request. hold=True: results stay in server staging (see result/release)."""
        r = np.ascontiguousarray(rays, dtype=np.float32)
        assert r.ndim == 2 and r.shape[1] == 8
        if hits is None and not hold:
            hits = np.empty((len(r), 4), dtype=np.int32)
        if hits is not None:
            assert hits.dtype == np.int32 and hits.shape == (len(r), 4) and hits.flags.c_contiguous
        rid = ctypes.c_uint64()
        _check(lib().hvf_server_submit(self._h, vol_id, r.ctypes.data if len(r) else None, len(r),
                                       hits.ctypes.data if (hits is not None and len(r)) else None,
                                       ctypes.byref(rid)))
        self._keep[rid.value] = (r, hits)
        return rid.value

    def result(self, req_id: int) -> np.ndarray:
        """View of a held request's hits in server staging (valid until release)."""
        p = ctypes.c_void_p()
        _check(lib().hvf_server_result(self._h, req_id, ctypes.byref(p)))
        n = len(self._keep[req_id][0])
        if n == 0:
            return np.zeros((0, 4), np.int32)
        buf = (ctypes.c_int32 * (4 * n)).from_address(p.value)
        return np.frombuffer(buf, dtype=np.int32).reshape(n, 4)

    def release(self, req_id: int):
        _check(lib().hvf_server_release(self._h, req_id))
        self._keep.pop(req_id, None)

    def poll(self, req_id: int):
        done, lat = ctypes.c_int(), ctypes.c_double()
        _check(lib().hvf_server_poll(self._h, req_id, ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def wait(self, req_id: int):
        """Block until done; returns (hits, latency_ms). Held requests: (None, latency)."""
        lat = ctypes.c_double()
        _check(lib().hvf_server_wait(self._h, req_id, ctypes.byref(lat)))
        r, h = self._keep[req_id]
        if h is not None:
            self._keep.pop(req_id)
        return h, lat.value

    def fail_steps(self, n: int):
        """Testing: make the next n steps fail at launch (hvf_server_fail_steps)."""
        _check(lib().hvf_server_fail_steps(self._h, n))

    def drain(self):
        _check(lib().hvf_server_drain(self._h))

    def stats(self) -> dict:
        st = hvf_serve_stats()
        _check(lib().hvf_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in hvf_serve_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().hvf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols() -> list[str]:
    """Names declared in include/hvf.h (for the export check)."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "hvf.h")
    src = open(hdr).read()
    return sorted(set(re.findall(r"\b(hvf_[a-z_0-9]+)\s*\(", src)))
