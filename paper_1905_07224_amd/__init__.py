"""Two-pass parallel gzip decompression on AMD Instinct MI355X (gfx950).

Python binding over the C ABI of ``libgzgpu.so`` (declared in
``include/gzgpu.h``).  It only marshals arguments: torch tensors provide the
device memory (compressed input, output, workspace) and the stream; every
step of the decompression runs in the library's HIP kernels.  There is no CPU
fallback: without the built library every call raises.

The method (Kerbiriou & Chikhi, Section VI-C): cut the compressed payload into
chunks, find a block start in each (Section VI-A, Appendix A), decode each
chunk with a context of 32768 unique placeholder symbols, resolve the 32 KiB
windows chunk after chunk, and replace every placeholder by its byte.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

__all__ = ["GzError", "Plan", "BatchPlan", "decompress", "decompress_batch", "lib", "Opts", "LIB_PATH"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgzgpu.so")

GZ_OK, GZ_E_ARG, GZ_E_HEADER, GZ_E_UNSUPPORTED, GZ_E_DATA, GZ_E_CAPACITY = 0, -1, -2, -3, -4, -5
GZ_E_CRC, GZ_E_SIZE, GZ_E_HIP, GZ_E_NOT_READY = -6, -7, -9, -10
NONE = (1 << 64) - 1


class GzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gzgpu error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("chunk_bytes", C.c_uint64), ("sym_factor", C.c_uint32), ("window_syms", C.c_uint32),
                ("scan_groups", C.c_uint32), ("inflate_waves_per_cu", C.c_uint32), ("waves_per_chunk", C.c_uint32),
                ("timing", C.c_uint32), ("confirm_decode", C.c_uint32), ("binary", C.c_uint32),
                ("tuned", C.c_uint32), ("start_types", C.c_uint32), ("reserved", C.c_uint32 * 2)]


class Job(C.Structure):
    _fields_ = [("d_comp", C.c_void_p), ("comp_len", C.c_uint64), ("n_chunks", C.c_int32), ("pad", C.c_int32),
                ("d_out", C.c_void_p), ("out_cap", C.c_uint64)]


class Info(C.Structure):
    _fields_ = [("ws_bytes", C.c_uint64), ("payload_start", C.c_uint64), ("payload_end", C.c_uint64),
                ("n_files", C.c_uint32), ("n_chunks", C.c_uint32), ("crc32", C.c_uint32), ("isize", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_chunks", C.c_uint32), ("out_len", C.c_uint64),
                ("out_needed", C.c_uint64), ("ws_needed", C.c_uint64), ("n_nonempty", C.c_uint32),
                ("n_repairs", C.c_uint32), ("n_extended", C.c_uint32), ("n_retries", C.c_uint32),
                ("n_syms", C.c_uint64), ("n_placeholders", C.c_uint64), ("n_blocks", C.c_uint64),
                ("crc32", C.c_uint32), ("inflate_waves", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("max_inflight", C.c_uint32), ("max_batch", C.c_uint32), ("opts", Opts)]


class Done(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("pad", C.c_uint32), ("out_len", C.c_uint64),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class ServerInfo(C.Structure):
    _fields_ = [("queued", C.c_uint32), ("running", C.c_uint32), ("finished_unread", C.c_uint32),
                ("mem_waited", C.c_uint32), ("batches", C.c_uint64), ("arena_bytes", C.c_uint64),
                ("arena_used", C.c_uint64), ("arena_peak", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("resident", C.c_uint64), ("resident_peak", C.c_uint64), ("now", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class StreamInfo(C.Structure):
    _fields_ = [("ws_bytes", C.c_uint64), ("out_bytes", C.c_uint64), ("segment_bytes", C.c_uint64),
                ("payload_start", C.c_uint64), ("payload_end", C.c_uint64), ("crc32", C.c_uint32),
                ("isize", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SegmentResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("done", C.c_uint32), ("out_len", C.c_uint64), ("out_total", C.c_uint64),
                ("start_bit", C.c_uint64), ("end_bit", C.c_uint64), ("out_needed", C.c_uint64),
                ("ws_needed", C.c_uint64), ("crc32", C.c_uint32), ("n_chunks", C.c_uint32),
                ("n_repairs", C.c_uint32), ("n_retries", C.c_uint32), ("member", C.c_uint32),
                ("member_done", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Checkpoint(C.Structure):
    _fields_ = [("bit", C.c_uint64), ("out_total", C.c_uint64), ("member_out", C.c_uint64),
                ("member", C.c_uint32), ("pad", C.c_uint32), ("crc32", C.c_uint32), ("valid", C.c_uint32),
                ("done", C.c_uint32), ("flags", C.c_uint32), ("window", C.c_uint8 * 32768)]


_lib = None

EXPORTS = ["gz_plan", "gz_plan_batch", "gz_plan_info", "gz_decompress", "gz_decompress_batch", "gz_result_get",
           "gz_chunk_table", "gz_debug_layout", "gz_plan_destroy", "gz_strerror", "gz_device_info", "gz_pass_times",
           "gz_pass_name", "gz_decompress_graph", "gz_autotune", "gz_server_create", "gz_server_submit",
           "gz_server_poll", "gz_server_stats", "gz_server_destroy", "gz_stream_open", "gz_stream_get_info",
           "gz_stream_next", "gz_stream_wait", "gz_stream_checkpoint", "gz_stream_resume", "gz_stream_destroy",
           "gz_plan_probes", "gz_find_blocks", "gz_probe_starts", "gz_stream_open_at", "gz_count_byte",
           "gz_plan_bgzf", "gz_chunk_stats", "gz_decompress_static", "gz_extract_dna_ws", "gz_extract_dna",
           "gz_decompress_members"]
GZ_N_PASSES = N_PASSES = 13
GZ_SCRATCH_BYTES = 256 << 20  # static workspace of gz_decompress_static, per GPU
# defaults of gz_opts (include/gzgpu.h)
DEFAULT_CHUNK_BYTES = 40 << 10
GZ_START_STORED = 2  # opts.start_types: stored blocks as chunk starts
DEFAULT_WINDOW = 512


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is the only implementation)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64 = C.c_void_p, C.c_int, C.c_uint64
        L.gz_plan.argtypes = [C.POINTER(vp), vp, C.c_size_t, i32, C.POINTER(Opts)]
        L.gz_plan_batch.argtypes = [C.POINTER(vp), C.POINTER(Job), i32, C.POINTER(Opts)]
        L.gz_plan_info.argtypes = [vp, C.POINTER(Info)]
        L.gz_decompress.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
        L.gz_decompress_batch.argtypes = [vp, vp, C.c_size_t, vp]
        L.gz_result_get.argtypes = [vp, i32, C.POINTER(Result)]
        L.gz_chunk_table.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.gz_chunk_stats.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.gz_decompress_static.argtypes = [vp, vp, C.c_size_t, vp]
        L.gz_debug_layout.argtypes = [vp, i32, vp, vp, C.POINTER(vp), C.POINTER(vp)]
        L.gz_plan_destroy.argtypes = [vp]
        L.gz_plan_destroy.restype = None
        L.gz_strerror.argtypes = [i32]
        L.gz_strerror.restype = C.c_char_p
        L.gz_device_info.argtypes = [i32, C.POINTER(i32), C.POINTER(i32)]
        L.gz_pass_times.argtypes = [vp, C.POINTER(C.c_float), i32]
        L.gz_decompress_graph.argtypes = [vp, vp, C.c_size_t, vp]
        L.gz_autotune.argtypes = [vp, C.c_size_t, vp, C.c_size_t, vp, C.c_size_t, vp, C.POINTER(Opts),
                                  C.POINTER(u64)]
        L.gz_server_create.argtypes = [C.POINTER(vp), C.POINTER(ServerOpts)]
        L.gz_server_submit.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, u64]
        L.gz_server_poll.argtypes = [vp, C.POINTER(Done), i32]
        L.gz_server_stats.argtypes = [vp, C.POINTER(ServerInfo)]
        L.gz_server_destroy.argtypes = [vp]
        L.gz_server_destroy.restype = None
        L.gz_pass_name.argtypes = [i32]
        L.gz_pass_name.restype = C.c_char_p
        L.gz_stream_open.argtypes = [C.POINTER(vp), vp, C.c_size_t, u64, C.POINTER(Opts)]
        L.gz_stream_get_info.argtypes = [vp, C.POINTER(StreamInfo)]
        L.gz_stream_next.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
        L.gz_stream_wait.argtypes = [vp, C.POINTER(SegmentResult)]
        L.gz_stream_checkpoint.argtypes = [vp, C.POINTER(Checkpoint)]
        L.gz_stream_resume.argtypes = [vp, C.POINTER(Checkpoint)]
        L.gz_stream_destroy.argtypes = [vp]
        L.gz_stream_destroy.restype = None
        L.gz_plan_probes.argtypes = [C.POINTER(vp), vp, C.c_size_t, vp, i32, u64, C.POINTER(Opts)]
        L.gz_find_blocks.argtypes = [vp, vp, C.c_size_t, vp]
        L.gz_probe_starts.argtypes = [vp, vp, vp]
        L.gz_stream_open_at.argtypes = [C.POINTER(vp), vp, C.c_size_t, u64, C.c_uint32, u64, C.POINTER(Opts)]
        L.gz_count_byte.argtypes = [vp, u64, C.c_uint32, u64, u64, vp, u64, vp]
        L.gz_decompress_members.argtypes = [vp, C.c_size_t, vp, C.c_size_t, vp, C.c_size_t, C.POINTER(Opts), vp,
                                            C.POINTER(u64), C.POINTER(C.c_uint32), C.POINTER(u64)]
        L.gz_extract_dna_ws.argtypes = [u64]
        L.gz_extract_dna_ws.restype = u64
        L.gz_extract_dna.argtypes = [vp, u64, C.c_uint32, C.c_uint32, C.c_uint32, vp, u64, vp, vp, C.c_uint32,
                                     C.c_uint32, vp, vp, C.c_size_t, vp]
        L.gz_plan_bgzf.argtypes = [C.POINTER(vp), vp, vp, C.c_size_t, vp, C.c_size_t, C.POINTER(Opts),
                                   C.POINTER(u64), C.POINTER(C.c_uint32)]
        for name in EXPORTS:
            if name not in ("gz_plan_destroy", "gz_strerror", "gz_pass_name", "gz_server_destroy",
                            "gz_stream_destroy", "gz_extract_dna_ws"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(code: int):
    if code != GZ_OK:
        raise GzError(code, lib().gz_strerror(code).decode())


def _opts(**kw) -> Opts:
    o = Opts()
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _as_device_bytes(comp, device=None) -> torch.Tensor:
    if isinstance(comp, torch.Tensor):
        t = comp
    else:
        t = torch.frombuffer(bytearray(comp), dtype=torch.uint8)
    if not t.is_cuda:
        t = t.to(device or "cuda", non_blocking=False)
    if t.dtype != torch.uint8 or not t.is_contiguous():
        raise ValueError("compressed input must be a contiguous uint8 tensor")
    return t


def _out_guess(isize: int, comp_len: int) -> int:
    # ISIZE is the length mod 2^32; text never decodes to much less than its
    # compressed size, so the smallest value at or above that bound is the guess
    floor = max(0, int(0.98 * (comp_len - 64)))
    n = isize
    while n < floor:
        n += 1 << 32
    return n


class Plan:
    """A one-file plan: chunk layout, workspace, and the launch sequence."""

    def __init__(self, comp, n_chunks: int = 0, **opts):
        self.comp = _as_device_bytes(comp)
        self.device = self.comp.device
        self.opts = _opts(**opts)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().gz_plan(C.byref(self._h), C.c_void_p(self.comp.data_ptr()), self.comp.numel(),
                                 int(n_chunks), C.byref(self.opts)))
        self.info = Info()
        _check(lib().gz_plan_info(self._h, C.byref(self.info)))
        self.ws = None
        self._graph_out = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gz_plan_destroy(h)
            self._h = C.c_void_p()

    @property
    def n_chunks(self) -> int:
        return self.info.n_chunks

    def workspace(self) -> torch.Tensor:
        if self.ws is None or self.ws.numel() < self.info.ws_bytes:
            self.ws = torch.empty(self.info.ws_bytes, dtype=torch.uint8, device=self.device)
        return self.ws

    def launch(self, out: torch.Tensor | None, stream=None, workspace: torch.Tensor | None = None):
        """Enqueue the decompression on `stream`; `workspace` (optional) is a
        caller's device buffer used instead of the plan's own."""
        ws = self.workspace() if workspace is None else workspace
        optr = C.c_void_p(out.data_ptr()) if out is not None and out.numel() else C.c_void_p()
        ocap = out.numel() if out is not None else 0
        with torch.cuda.device(self.device):
            _check(lib().gz_decompress(self._h, optr, ocap, C.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_handle(stream)))

    def launch_static(self, out: torch.Tensor | None, stream=None):
        """Like launch(), with the library's static per-GPU workspace
        (gz_decompress_static: nothing is allocated)."""
        optr = C.c_void_p(out.data_ptr()) if out is not None and out.numel() else C.c_void_p()
        ocap = out.numel() if out is not None else 0
        with torch.cuda.device(self.device):
            _check(lib().gz_decompress_static(self._h, optr, ocap, _stream_handle(stream)))

    def launch_graph(self, out: torch.Tensor | None, stream):
        """Like launch(), through the plan's captured HIP graph (captured again
        when the output or the workspace changes); `stream` must not be the
        null stream."""
        ws = self.workspace()
        if self._graph_out is not out:
            # the output enters the plan through the eager entry point, once
            self._graph_out = out
            self.launch(out, stream)
            self.result()
        with torch.cuda.device(self.device):
            _check(lib().gz_decompress_graph(self._h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))

    def result(self, file: int = 0) -> Result:
        r = Result()
        _check(lib().gz_result_get(self._h, file, C.byref(r)))
        return r

    def pass_times(self):
        """{pass name: ms} of the last launch (needs timing=1 in the options)."""
        return _pass_times(self._h)

    def chunk_table(self, file: int = 0):
        import numpy as np

        n = self.info.n_chunks
        arrs = {k: np.zeros(n, dtype=np.uint64) for k in ("start", "cand", "end", "len", "out_off")}
        st = np.zeros(n, dtype=np.int32)
        fl = np.zeros(n, dtype=np.uint32)
        p = lambda a: C.c_void_p(a.ctypes.data)  # noqa: E731
        _check(lib().gz_chunk_table(self._h, file, p(arrs["start"]), p(arrs["cand"]), p(arrs["end"]),
                                    p(arrs["len"]), p(arrs["out_off"]), p(st), p(fl)))
        arrs["status"] = st
        arrs["flags"] = fl
        return arrs

    def chunk_stats(self, file: int = 0):
        """Per-chunk statistics (gz_chunk_stats): codes, placeholders, blocks,
        the static-check candidate and the block-start search's stage counts."""
        import numpy as np

        n = self.info.n_chunks
        a = {k: np.zeros(n, dtype=np.uint64) for k in ("n_syms", "n_placeholders", "scan_cand")}
        a.update({k: np.zeros(n, dtype=np.uint32) for k in ("n_blocks", "stage1", "stage2", "trial_rej",
                                                              "confirm_rej")})
        p = lambda x: C.c_void_p(x.ctypes.data)  # noqa: E731
        _check(lib().gz_chunk_stats(self._h, file, p(a["n_syms"]), p(a["n_placeholders"]), p(a["n_blocks"]),
                                    p(a["scan_cand"]), p(a["stage1"]), p(a["stage2"]), p(a["trial_rej"]),
                                    p(a["confirm_rej"])))
        return a

    def symbols(self, chunk: int, length: int) -> torch.Tensor:
        """The chunk's 16-bit symbols in the workspace (a view; valid until the next launch)."""
        import numpy as np

        n = self.info.n_chunks
        off = np.zeros(n, dtype=np.uint64)
        wi = np.zeros(n, dtype=np.uint64)
        sb, wb = C.c_void_p(), C.c_void_p()
        _check(lib().gz_debug_layout(self._h, 0, C.c_void_p(off.ctypes.data), C.c_void_p(wi.ctypes.data),
                                     C.byref(sb), C.byref(wb)))
        base = (sb.value - self.ws.data_ptr()) // 2 + int(off[chunk])
        return self.ws.view(torch.int16)[base:base + length].view(torch.uint16) if hasattr(torch, "uint16") \
            else self.ws.view(torch.int16)[base:base + length]

    def window(self, chunk: int) -> torch.Tensor:
        import numpy as np

        n = self.info.n_chunks
        off = np.zeros(n, dtype=np.uint64)
        wi = np.zeros(n, dtype=np.uint64)
        sb, wb = C.c_void_p(), C.c_void_p()
        _check(lib().gz_debug_layout(self._h, 0, C.c_void_p(off.ctypes.data), C.c_void_p(wi.ctypes.data),
                                     C.byref(sb), C.byref(wb)))
        base = wb.value - self.ws.data_ptr() + 32768 * int(wi[chunk])
        return self.ws[base:base + 32768]

    def run(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Decompress into `out` (allocated when None); raises GzError on any failure."""
        for _ in range(4):
            if out is None:
                out = torch.empty(_out_guess(self.info.isize, self.comp.numel()), dtype=torch.uint8,
                                  device=self.device)
            self.launch(out, stream)
            r = self.result()
            if r.status == GZ_E_CAPACITY and r.ws_needed:
                # a chunk produced more symbols than planned: re-plan with room for it
                factor = max(self.opts.sym_factor or 8, 8)
                while True:
                    factor *= 4
                    self.opts.sym_factor = factor
                    lib().gz_plan_destroy(self._h)
                    self._h = C.c_void_p()
                    _check(lib().gz_plan(C.byref(self._h), C.c_void_p(self.comp.data_ptr()), self.comp.numel(),
                                         int(self.info.n_chunks), C.byref(self.opts)))
                    _check(lib().gz_plan_info(self._h, C.byref(self.info)))
                    if self.info.ws_bytes >= r.ws_needed or factor > 4096:
                        break
                continue
            if r.status == GZ_E_CAPACITY and r.out_needed > out.numel():
                out = torch.empty(r.out_needed, dtype=torch.uint8, device=self.device)
                continue
            _check(r.status)
            return out[: r.out_len]
        raise GzError(GZ_E_CAPACITY, "capacity retries exhausted")


def _pass_times(h):
    buf = (C.c_float * N_PASSES)()
    n = lib().gz_pass_times(h, buf, N_PASSES)
    if n < 0:
        _check(n)
    return {lib().gz_pass_name(i).decode(): float(buf[i]) for i in range(n)}


def decompress(comp, n_chunks: int = 0, out=None, stream=None, **opts) -> torch.Tensor:
    """Decompress one gzip member held in a uint8 tensor (or bytes) on the GPU."""
    return Plan(comp, n_chunks, **opts).run(out, stream)


class BatchPlan:
    """Many files decoded by one launch sequence (one launch per pass)."""

    def __init__(self, comps, n_chunks=0, outs=None, **opts):
        self.comps = [_as_device_bytes(c) for c in comps]
        self.device = self.comps[0].device
        self.opts = _opts(**opts)
        nc = n_chunks if isinstance(n_chunks, (list, tuple)) else [n_chunks] * len(self.comps)
        self.n_chunks_req = list(nc)
        self.outs = outs
        self._h = C.c_void_p()
        self._make(outs)

    def _make(self, outs):
        n = len(self.comps)
        jobs = (Job * n)()
        self._isizes = []
        for i, c in enumerate(self.comps):
            jobs[i].d_comp = c.data_ptr()
            jobs[i].comp_len = c.numel()
            jobs[i].n_chunks = int(self.n_chunks_req[i])
            if outs is not None:
                jobs[i].d_out = outs[i].data_ptr()
                jobs[i].out_cap = outs[i].numel()
        if self._h.value:
            lib().gz_plan_destroy(self._h)
            self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().gz_plan_batch(C.byref(self._h), jobs, n, C.byref(self.opts)))
        self.info = Info()
        _check(lib().gz_plan_info(self._h, C.byref(self.info)))
        self.ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gz_plan_destroy(h)
            self._h = C.c_void_p()

    def workspace(self) -> torch.Tensor:
        if self.ws is None or self.ws.numel() < self.info.ws_bytes:
            self.ws = torch.empty(self.info.ws_bytes, dtype=torch.uint8, device=self.device)
        return self.ws

    def launch(self, stream=None):
        ws = self.workspace()
        with torch.cuda.device(self.device):
            _check(lib().gz_decompress_batch(self._h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))

    def launch_graph(self, stream):
        """Like launch(), through the plan's captured HIP graph; `stream` must
        not be the null stream."""
        ws = self.workspace()
        with torch.cuda.device(self.device):
            _check(lib().gz_decompress_graph(self._h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))

    def result(self, file: int) -> Result:
        r = Result()
        _check(lib().gz_result_get(self._h, file, C.byref(r)))
        return r

    def pass_times(self):
        return _pass_times(self._h)


def _isize_of(t: torch.Tensor) -> int:
    tail = t[-4:].cpu().numpy().tobytes()
    return int.from_bytes(tail, "little")


def decompress_batch(comps, n_chunks=0, stream=None, **opts):
    """Decompress several gzip files with one launch per pass; returns a list of tensors."""
    comps = [_as_device_bytes(c) for c in comps]
    outs = [torch.empty(_out_guess(_isize_of(c), c.numel()), dtype=torch.uint8, device=c.device) for c in comps]
    bp = BatchPlan(comps, n_chunks, outs, **opts)
    for _ in range(4):
        bp.launch(stream)
        res = [bp.result(i) for i in range(len(comps))]
        redo = False
        for i, r in enumerate(res):
            if r.status == GZ_E_CAPACITY and r.ws_needed:
                bp.opts.sym_factor = max(bp.opts.sym_factor or 8, 8) * 8
                redo = True
            elif r.status == GZ_E_CAPACITY and r.out_needed > outs[i].numel():
                outs[i] = torch.empty(r.out_needed, dtype=torch.uint8, device=comps[i].device)
                redo = True
        if redo:
            bp._make(outs)
            continue
        for r in res:
            _check(r.status)
        return [o[: r.out_len] for o, r in zip(outs, res)]
    raise GzError(GZ_E_CAPACITY, "capacity retries exhausted")


def autotune(comp, out: torch.Tensor | None = None, stream=None, **opts) -> dict:
    """Tuned options (chunk_bytes, window_syms) for this input, from
    gz_autotune: every candidate is timed on the input itself, and the choice
    is cached per device and input class for the process."""
    comp = _as_device_bytes(comp)
    base = _opts(**opts)
    need = C.c_uint64(0)
    with torch.cuda.device(comp.device):
        _check(lib().gz_autotune(C.c_void_p(comp.data_ptr()), comp.numel(), None, 0, None, 0, None, C.byref(base),
                                 C.byref(need)))
        if out is None:
            info_plan = Plan(comp, 0, **opts)
            out = torch.empty(_out_guess(info_plan.info.isize, comp.numel()), dtype=torch.uint8, device=comp.device)
            del info_plan
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=comp.device)
        best = _opts(**opts)
        _check(lib().gz_autotune(C.c_void_p(comp.data_ptr()), comp.numel(), C.c_void_p(out.data_ptr()), out.numel(),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream), C.byref(best), None))
    return {"chunk_bytes": int(best.chunk_bytes), "window_syms": int(best.window_syms)}


class Server:
    """The serving loop of gz_server_*: submit jobs (device tensors), poll for
    finished ones.  The tensors of a job are held until it is reported done.
    The workspace arena (arena_bytes, default: the budget) is a torch tensor
    owned here and handed to the library."""

    def __init__(self, budget_bytes: int = 0, max_inflight: int = 0, max_batch: int = 0, device=None,
                 arena_bytes: int = 0, **opts):
        self.device = torch.device(device or "cuda:0")
        budget_bytes = budget_bytes or (96 << 30)
        arena_bytes = arena_bytes or budget_bytes
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        o = ServerOpts()
        o.arena = C.c_void_p(self.arena.data_ptr())
        o.arena_bytes = arena_bytes
        o.budget_bytes = budget_bytes
        o.max_inflight = max_inflight
        o.max_batch = max_batch
        o.opts = _opts(**opts)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().gz_server_create(C.byref(self._h), C.byref(o)))
        self._held = {}
        self._buf = (Done * 256)()

    def submit(self, comp: torch.Tensor, out: torch.Tensor, tag: int):
        with torch.cuda.device(self.device):
            _check(lib().gz_server_submit(self._h, C.c_void_p(comp.data_ptr()), comp.numel(),
                                          C.c_void_p(out.data_ptr()), out.numel(), int(tag)))
        self._held[int(tag)] = (comp, out)

    def poll(self):
        """Finished jobs (dicts of gz_done), possibly none; never waits."""
        res = []
        while True:
            with torch.cuda.device(self.device):
                n = lib().gz_server_poll(self._h, self._buf, len(self._buf))
            if n < 0:
                _check(n)
            for i in range(n):
                d = self._buf[i].as_dict()
                self._held.pop(d["tag"], None)
                res.append(d)
            if n < len(self._buf):
                return res

    def stats(self) -> dict:
        i = ServerInfo()
        _check(lib().gz_server_stats(self._h, C.byref(i)))
        return i.as_dict()

    def close(self):
        if self._h.value:
            lib().gz_server_destroy(self._h)
            self._h = C.c_void_p()
        self._held.clear()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gz_server_destroy(h)
            self._h = C.c_void_p()


class Stream:
    """Bounded-memory decoding of one gzip member in segments (gz_stream_*).

    Each segment() call decodes the next segment into an output buffer that
    is reused (a view of it is returned: copy it before the next call) and a
    workspace sized for one segment; the carried window stays on the device.
    checkpoint() / resume() save and restore the position."""

    def __init__(self, comp, segment_bytes: int = 0, stream=None, at_bit: int | None = None, marker: int = 0,
                 **opts):
        """at_bit: start at this block start inside the member (random access)
        with an undetermined context of `marker` bytes."""
        self.comp = _as_device_bytes(comp)
        self.device = self.comp.device
        self.stream = stream
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            if at_bit is None:
                _check(lib().gz_stream_open(C.byref(self._h), C.c_void_p(self.comp.data_ptr()), self.comp.numel(),
                                            int(segment_bytes), C.byref(_opts(**opts))))
            else:
                _check(lib().gz_stream_open_at(C.byref(self._h), C.c_void_p(self.comp.data_ptr()),
                                               self.comp.numel(), int(at_bit), int(marker), int(segment_bytes),
                                               C.byref(_opts(**opts))))
        self._ws = None
        self._out = None
        self._info = None
        self.done = False
        self.last = None

    def info(self) -> dict:
        i = StreamInfo()
        with torch.cuda.device(self.device):
            _check(lib().gz_stream_get_info(self._h, C.byref(i)))
        return i.as_dict()

    def _buffers(self, ws_bytes: int, out_bytes: int):
        if self._ws is None or self._ws.numel() < ws_bytes:
            self._ws = None
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        if self._out is None or self._out.numel() < out_bytes:
            self._out = None
            self._out = torch.empty(max(out_bytes, 1), dtype=torch.uint8, device=self.device)

    def segment(self, retries: int = 4) -> torch.Tensor:
        """Decode the next segment; returns its bytes (a view of the reused
        output buffer).  Raises GzError on a data error."""
        if self.done:
            raise GzError(GZ_E_ARG, "the member is finished")
        for _ in range(retries + 1):
            if self._info is None or (self.last is not None and self.last["status"] == GZ_E_CAPACITY):
                self._info = self.info()
            info = self._info
            out_need = info["out_bytes"]
            if self.last is not None and self.last["status"] == GZ_E_CAPACITY:
                out_need = max(out_need, self.last["out_needed"])
            self._buffers(info["ws_bytes"], out_need)
            with torch.cuda.device(self.device):
                _check(lib().gz_stream_next(self._h, C.c_void_p(self._out.data_ptr()), self._out.numel(),
                                            C.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                            _stream_handle(self.stream)))
                r = SegmentResult()
                _check(lib().gz_stream_wait(self._h, C.byref(r)))
            self.last = r.as_dict()
            if r.status == GZ_OK:
                self.done = bool(r.done)
                return self._out[:r.out_len]
            if r.status != GZ_E_CAPACITY:
                _check(r.status)
        _check(GZ_E_CAPACITY)

    def __iter__(self):
        while not self.done:
            yield self.segment()

    def checkpoint(self) -> Checkpoint:
        cp = Checkpoint()
        with torch.cuda.device(self.device):
            _check(lib().gz_stream_checkpoint(self._h, C.byref(cp)))
        return cp

    def resume(self, cp: Checkpoint):
        with torch.cuda.device(self.device):
            _check(lib().gz_stream_resume(self._h, C.byref(cp)))
        self.done = bool(cp.done)
        self.last = None

    def close(self):
        if self._h.value:
            lib().gz_stream_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.gz_stream_destroy(h)
            self._h = C.c_void_p()


def decompress_stream(comp, segment_bytes: int = 0, stream=None, **opts) -> torch.Tensor:
    """The member decoded segment by segment, concatenated (for tests: the
    bounded-memory use keeps only one segment at a time)."""
    s = Stream(comp, segment_bytes, stream=stream, **opts)
    parts = [seg.clone() for seg in s]
    s.close()
    return torch.cat(parts) if parts else torch.empty(0, dtype=torch.uint8, device=s.device)


def find_blocks(comp, bits, range_bytes: int = 0, stream=None, **opts):
    """Block starts at or after each bit offset (gz_plan_probes /
    gz_find_blocks): a list of ints, None where no start passed the checks
    within range_bytes; and the candidates each probe rejected."""
    import numpy as np

    comp = _as_device_bytes(comp)
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint64))
    h = C.c_void_p()
    with torch.cuda.device(comp.device):
        _check(lib().gz_plan_probes(C.byref(h), C.c_void_p(comp.data_ptr()), comp.numel(),
                                    C.c_void_p(b.ctypes.data), int(b.size), int(range_bytes),
                                    C.byref(_opts(**opts))))
        try:
            info = Info()
            _check(lib().gz_plan_info(h, C.byref(info)))
            ws = torch.empty(info.ws_bytes, dtype=torch.uint8, device=comp.device)
            _check(lib().gz_find_blocks(h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
            starts = np.zeros(b.size, dtype=np.uint64)
            rej = np.zeros(b.size, dtype=np.uint32)
            _check(lib().gz_probe_starts(h, C.c_void_p(starts.ctypes.data), C.c_void_p(rej.ctypes.data)))
        finally:
            lib().gz_plan_destroy(h)
    return [None if int(x) == NONE else int(x) for x in starts], [int(x) for x in rej]


def count_byte(buf: torch.Tensor, value: int, window: int, counts: torch.Tensor, first: int = 0, stream=None):
    """counts[(first + i) // window] += (buf[i] == value) on the device (gz_count_byte);
    counts is an int64 device tensor."""
    if counts.dtype != torch.int64 or not counts.is_cuda or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous int64 device tensor")
    with torch.cuda.device(buf.device):
        _check(lib().gz_count_byte(C.c_void_p(buf.data_ptr()), buf.numel(), int(value), int(first), int(window),
                                   C.c_void_p(counts.data_ptr()), counts.numel(), _stream_handle(stream)))


def decompress_members(comp, out: torch.Tensor, stream=None, **opts):
    """Concatenated gzip members into `out` (gz_decompress_members: each
    member by the whole parallel path, members one after another; waits).
    Returns (bytes written, members).  Raises GzError on failure."""
    comp = _as_device_bytes(comp)
    o = _opts(**opts)
    need = C.c_uint64(0)
    n_out, n_mem = C.c_uint64(0), C.c_uint32(0)
    with torch.cuda.device(comp.device):
        _check(lib().gz_decompress_members(C.c_void_p(comp.data_ptr()), comp.numel(), None, 0, None, 0, C.byref(o),
                                           None, None, None, C.byref(need)))
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=comp.device)
        _check(lib().gz_decompress_members(C.c_void_p(comp.data_ptr()), comp.numel(), C.c_void_p(out.data_ptr()),
                                           out.numel(), C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(o),
                                           _stream_handle(stream), C.byref(n_out), C.byref(n_mem), C.byref(need)))
    return int(n_out.value), int(n_mem.value)


class DnaSeq(C.Structure):
    _fields_ = [("start", C.c_uint64), ("len", C.c_uint32), ("n_undetermined", C.c_uint32)]


DNA_SEQ_DTYPE = [(f, np_t) for (f, _), np_t in zip(DnaSeq._fields_, ("<u8", "<u4", "<u4"))]


def extract_dna(buf: torch.Tensor, marker: int | None = None, min_len: int = 1, bounds=None, threshold: int = 1,
                max_seqs: int | None = None, stream=None):
    """DNA-like sequences of a partly undetermined text (gz_extract_dna,
    Appendix B).  buf: a uint8 device tensor whose value `marker` is
    undetermined, or 16-bit symbols (int16/uint16) whose values of 256 and
    above are.  bounds: n_ranges + 1 ascending positions, or None.  Returns
    (numpy array of gz_dna_seq records, total found, numpy array of
    (sequences, with undetermined, resolved) per range or None)."""
    import numpy as np

    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    elem = buf.element_size()
    if elem not in (1, 2):
        raise ValueError("buf must hold bytes or 16-bit symbols")
    if elem == 1 and marker is None:
        raise ValueError("a byte buffer needs its marker value")
    n = buf.numel()
    dev = buf.device
    if max_seqs is None:
        max_seqs = (n + 2) // 3
    rec_bytes = C.sizeof(DnaSeq)
    seqs = torch.empty(max(1, max_seqs) * rec_bytes, dtype=torch.uint8, device=dev)
    n_seqs = torch.zeros(1, dtype=torch.int64, device=dev)
    nr = 0
    b = st = None
    if bounds is not None:
        b = torch.as_tensor(np.asarray(bounds, dtype=np.int64)).to(dev)
        nr = b.numel() - 1
        st = torch.empty(max(1, 3 * nr), dtype=torch.int32, device=dev)
    ws_bytes = int(lib().gz_extract_dna_ws(n))
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    with torch.cuda.device(dev):
        h = _stream_handle(stream)
        _check(lib().gz_extract_dna(C.c_void_p(buf.data_ptr()), n, elem, int(marker or 0), int(min_len),
                                    C.c_void_p(seqs.data_ptr()), int(max_seqs), C.c_void_p(n_seqs.data_ptr()),
                                    C.c_void_p(b.data_ptr()) if b is not None else None, nr, int(threshold),
                                    C.c_void_p(st.data_ptr()) if st is not None else None,
                                    C.c_void_p(ws.data_ptr() + off), ws_bytes, h))
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
    total = int(n_seqs.item())
    k = min(total, max_seqs)
    rec = np.frombuffer(seqs[: rec_bytes * k].cpu().numpy().tobytes(), dtype=DNA_SEQ_DTYPE)
    stats = st[: 3 * nr].cpu().numpy().astype(np.int64).reshape(nr, 3) if st is not None else None
    return rec, total, stats


def undetermined_profile(comp, bit: int, window: int, marker: int = 0, segment_bytes: int = 0,
                         max_out: int | None = None, range_bytes: int = 0, **opts):
    """Random access at `bit` (Section IV): the first block start at or after
    it, then decoding to the end of the member (or max_out bytes) with an
    undetermined context.  Returns (block start, decoded bytes, undetermined
    bytes per window of `window` bytes as an int64 numpy array)."""
    comp = _as_device_bytes(comp)
    starts, _ = find_blocks(comp, [bit], range_bytes, **opts)
    if starts[0] is None:
        raise GzError(GZ_E_DATA, "no block start passed the checks in the probe's range")
    s = Stream(comp, segment_bytes, at_bit=starts[0], marker=marker, **opts)
    limit = max_out if max_out is not None else (1 << 62)
    cap = 1 << 16
    counts = torch.zeros(cap, dtype=torch.int64, device=comp.device)
    total = 0
    try:
        for part in s:
            part = part[: max(0, limit - total)]
            need = (total + part.numel() + window - 1) // window
            if need > counts.numel():
                grown = torch.zeros(max(need, 2 * counts.numel()), dtype=torch.int64, device=comp.device)
                grown[: counts.numel()] = counts
                counts = grown
            count_byte(part, marker, window, counts, first=total)
            total += part.numel()
            if total >= limit:
                break
    finally:
        s.close()
    torch.cuda.synchronize()
    n_win = (total + window - 1) // window
    return starts[0], total, counts[:n_win].cpu().numpy()


def decompress_bgzf(comp, stream=None, **opts) -> torch.Tensor:
    """A BGZF-style input decoded with one batch plan (gz_plan_bgzf): every
    member at once, outputs back to back.  Raises GzError on any member's
    failure."""
    host = comp if isinstance(comp, (bytes, bytearray)) else None
    dcomp = _as_device_bytes(comp)
    hbuf = None
    if host is not None:
        hbuf = (C.c_uint8 * len(host)).from_buffer_copy(bytes(host))
    n_out, n_mem = C.c_uint64(), C.c_uint32()
    h = C.c_void_p()
    with torch.cuda.device(dcomp.device):
        _check(lib().gz_plan_bgzf(C.byref(h), C.c_void_p(dcomp.data_ptr()), hbuf, dcomp.numel(), None, 0,
                                  C.byref(_opts(**opts)), C.byref(n_out), C.byref(n_mem)))
        lib().gz_plan_destroy(h)
        out = torch.empty(max(1, n_out.value), dtype=torch.uint8, device=dcomp.device)
        h = C.c_void_p()
        _check(lib().gz_plan_bgzf(C.byref(h), C.c_void_p(dcomp.data_ptr()), hbuf, dcomp.numel(),
                                  C.c_void_p(out.data_ptr()), out.numel(), C.byref(_opts(**opts)), C.byref(n_out),
                                  C.byref(n_mem)))
        try:
            info = Info()
            _check(lib().gz_plan_info(h, C.byref(info)))
            ws = torch.empty(info.ws_bytes, dtype=torch.uint8, device=dcomp.device)
            _check(lib().gz_decompress_batch(h, C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
            for f in range(n_mem.value):
                r = Result()
                _check(lib().gz_result_get(h, f, C.byref(r)))
                _check(r.status)
        finally:
            lib().gz_plan_destroy(h)
    return out[: n_out.value]
