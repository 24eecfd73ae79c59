"""Drive the device path's C ABI on the CPU through the test-side executor (tests/emu)."""
import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


class Opts(C.Structure):
    _fields_ = [("chunk_bytes", C.c_uint64), ("sym_factor", C.c_uint32), ("window_syms", C.c_uint32),
                ("scan_groups", C.c_uint32), ("inflate_waves_per_cu", C.c_uint32), ("waves_per_chunk", C.c_uint32),
                ("timing", C.c_uint32), ("confirm_decode", C.c_uint32), ("binary", C.c_uint32),
                ("tuned", C.c_uint32), ("start_types", C.c_uint32), ("reserved", C.c_uint32 * 2)]


class Info(C.Structure):
    _fields_ = [("ws_bytes", C.c_uint64), ("payload_start", C.c_uint64), ("payload_end", C.c_uint64),
                ("n_files", C.c_uint32), ("n_chunks", C.c_uint32), ("crc32", C.c_uint32), ("isize", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_chunks", C.c_uint32), ("out_len", C.c_uint64),
                ("out_needed", C.c_uint64), ("ws_needed", C.c_uint64), ("n_nonempty", C.c_uint32),
                ("n_repairs", C.c_uint32), ("n_extended", C.c_uint32), ("n_retries", C.c_uint32),
                ("n_syms", C.c_uint64), ("n_placeholders", C.c_uint64), ("n_blocks", C.c_uint64),
                ("crc32", C.c_uint32), ("inflate_waves", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GZEMU_LIB")
        if not path:
            import build as ebuild  # tests/emu/build.py

            path = ebuild.build()
        _lib = C.CDLL(path)
        vp = C.c_void_p
        _lib.gz_plan.argtypes = [C.POINTER(vp), vp, C.c_size_t, C.c_int, C.POINTER(Opts)]
        _lib.gz_plan_info.argtypes = [vp, C.POINTER(Info)]
        _lib.gz_decompress.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
        _lib.gz_result_get.argtypes = [vp, C.c_int, C.POINTER(Result)]
        _lib.gz_chunk_table.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        _lib.gz_chunk_stats.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.gz_plan_destroy.argtypes = [vp]
        _lib.gz_plan_destroy.restype = None
        _lib.emu_set_sync_limit.argtypes = [C.c_uint64]
    return _lib


def run(comp: bytes, n_chunks: int, out_cap=None, sync_limit=0, **opts):
    L = lib()
    L.emu_set_sync_limit(sync_limit)
    # the device path reads whole aligned dwords that hold input bytes; pad the
    # host copy so that those reads stay inside the allocation
    store = np.zeros(len(comp) + (-len(comp)) % 8, dtype=np.uint8)
    store[: len(comp)] = np.frombuffer(bytes(comp), dtype=np.uint8)
    buf = store[: len(comp)]
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = L.gz_plan(C.byref(h), C.c_void_p(buf.ctypes.data), buf.size, n_chunks, C.byref(o))
    if st != 0:
        return st, None, None, None
    info = Info()
    L.gz_plan_info(h, C.byref(info))
    raw_ws = np.zeros(info.ws_bytes + 512, dtype=np.uint8)
    off = (-raw_ws.ctypes.data) % 256
    ws = raw_ws[off:off + info.ws_bytes]
    if out_cap is None:
        out_cap = max(1, int(info.isize))
    out = np.zeros(out_cap, dtype=np.uint8)
    st = L.gz_decompress(h, C.c_void_p(out.ctypes.data), out_cap, C.c_void_p(ws.ctypes.data), ws.size, None)
    assert st == 0, st
    r = Result()
    L.gz_result_get(h, 0, C.byref(r))
    n = info.n_chunks
    tab = {k: np.zeros(n, dtype=np.uint64) for k in ("start", "cand", "end", "len", "out_off")}
    sts = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint32)
    p = lambda a: C.c_void_p(a.ctypes.data)  # noqa: E731
    L.gz_chunk_table(h, 0, p(tab["start"]), p(tab["cand"]), p(tab["end"]), p(tab["len"]), p(tab["out_off"]),
                     p(sts), p(fl))
    tab["status"], tab["flags"] = sts, fl
    for k in ("n_syms", "n_placeholders", "scan_cand"):
        tab[k] = np.zeros(n, dtype=np.uint64)
    for k in ("n_blocks", "stage1", "stage2", "trial_rej", "confirm_rej"):
        tab[k] = np.zeros(n, dtype=np.uint32)
    assert L.gz_chunk_stats(h, 0, p(tab["n_syms"]), p(tab["n_placeholders"]), p(tab["n_blocks"]), p(tab["scan_cand"]),
                            p(tab["stage1"]), p(tab["stage2"]), p(tab["trial_rej"]), p(tab["confirm_rej"])) == 0
    L.gz_plan_destroy(h)
    return r.status, out[: r.out_len].tobytes(), r, tab


class ServerOpts(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("max_inflight", C.c_uint32), ("max_batch", C.c_uint32), ("opts", Opts)]


class Done(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("pad", C.c_uint32), ("out_len", C.c_uint64),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_end", C.c_double)]


class ServerInfo(C.Structure):
    _fields_ = [("queued", C.c_uint32), ("running", C.c_uint32), ("finished_unread", C.c_uint32),
                ("mem_waited", C.c_uint32), ("batches", C.c_uint64), ("arena_bytes", C.c_uint64),
                ("arena_used", C.c_uint64), ("arena_peak", C.c_uint64), ("budget_bytes", C.c_uint64),
                ("resident", C.c_uint64), ("resident_peak", C.c_uint64), ("now", C.c_double)]


def server_lib():
    L = lib()
    vp = C.c_void_p
    L.gz_server_create.argtypes = [C.POINTER(vp), C.POINTER(ServerOpts)]
    L.gz_server_submit.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, C.c_uint64]
    L.gz_server_poll.argtypes = [vp, C.POINTER(Done), C.c_int]
    L.gz_server_stats.argtypes = [vp, C.POINTER(ServerInfo)]
    L.gz_server_destroy.argtypes = [vp]
    L.gz_server_destroy.restype = None
    return L


def padded(comp: bytes):
    """Host copy of a compressed input, padded so whole-dword reads stay inside."""
    store = np.zeros(len(comp) + (-len(comp)) % 8 + 8, dtype=np.uint8)
    store[: len(comp)] = np.frombuffer(bytes(comp), dtype=np.uint8)
    return store


class StreamInfo(C.Structure):
    _fields_ = [("ws_bytes", C.c_uint64), ("out_bytes", C.c_uint64), ("segment_bytes", C.c_uint64),
                ("payload_start", C.c_uint64), ("payload_end", C.c_uint64), ("crc32", C.c_uint32),
                ("isize", C.c_uint32)]


class SegmentResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("done", C.c_uint32), ("out_len", C.c_uint64), ("out_total", C.c_uint64),
                ("start_bit", C.c_uint64), ("end_bit", C.c_uint64), ("out_needed", C.c_uint64),
                ("ws_needed", C.c_uint64), ("crc32", C.c_uint32), ("n_chunks", C.c_uint32),
                ("n_repairs", C.c_uint32), ("n_retries", C.c_uint32), ("member", C.c_uint32),
                ("member_done", C.c_uint32)]


class Checkpoint(C.Structure):
    _fields_ = [("bit", C.c_uint64), ("out_total", C.c_uint64), ("member_out", C.c_uint64),
                ("member", C.c_uint32), ("pad", C.c_uint32), ("crc32", C.c_uint32), ("valid", C.c_uint32),
                ("done", C.c_uint32), ("flags", C.c_uint32), ("window", C.c_uint8 * 32768)]


def stream_lib():
    L = lib()
    vp = C.c_void_p
    L.gz_stream_open.argtypes = [C.POINTER(vp), vp, C.c_size_t, C.c_uint64, C.POINTER(Opts)]
    L.gz_stream_get_info.argtypes = [vp, C.POINTER(StreamInfo)]
    L.gz_stream_next.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
    L.gz_stream_wait.argtypes = [vp, C.POINTER(SegmentResult)]
    L.gz_stream_checkpoint.argtypes = [vp, C.POINTER(Checkpoint)]
    L.gz_stream_resume.argtypes = [vp, C.POINTER(Checkpoint)]
    L.gz_stream_destroy.argtypes = [vp]
    L.gz_stream_destroy.restype = None
    return L


def stream_run(comp: bytes, segment_bytes: int, resume=None, stop_after=None, **opts):
    """Decode through gz_stream_*: returns (segments: list of (SegmentResult
    dict, bytes, Checkpoint after it)).  resume: a Checkpoint to start from;
    stop_after: number of segments to run."""
    L = stream_lib()
    L.emu_set_sync_limit(3_000_000_000)
    store = padded(comp)
    buf = store[: len(comp)]
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = L.gz_stream_open(C.byref(h), C.c_void_p(buf.ctypes.data), buf.size, segment_bytes, C.byref(o))
    assert st == 0, st
    if resume is not None:
        assert L.gz_stream_resume(h, C.byref(resume)) == 0
    segs = []
    try:
        while stop_after is None or len(segs) < stop_after:
            info = StreamInfo()
            assert L.gz_stream_get_info(h, C.byref(info)) == 0
            raw_ws = np.zeros(info.ws_bytes + 512, dtype=np.uint8)
            off = (-raw_ws.ctypes.data) % 256
            ws = raw_ws[off:off + info.ws_bytes]
            out = np.zeros(max(1, info.out_bytes), dtype=np.uint8)
            st = L.gz_stream_next(h, C.c_void_p(out.ctypes.data), out.size, C.c_void_p(ws.ctypes.data), ws.size,
                                  None)
            if st != 0:
                segs.append(({"next_status": st}, b"", None))
                break
            r = SegmentResult()
            assert L.gz_stream_wait(h, C.byref(r)) == 0
            d = {k: getattr(r, k) for k, _ in r._fields_}
            cp = Checkpoint()
            assert L.gz_stream_checkpoint(h, C.byref(cp)) == 0
            segs.append((d, out[: r.out_len].tobytes() if r.status == 0 else b"", cp))
            if r.status != 0 or r.done:
                break
    finally:
        L.gz_stream_destroy(h)
    return segs


def probe_run(comp: bytes, bits, range_bytes: int, **opts):
    """gz_plan_probes + gz_find_blocks + gz_probe_starts; returns (starts, rejected)."""
    L = lib()
    vp = C.c_void_p
    L.gz_plan_probes.argtypes = [C.POINTER(vp), vp, C.c_size_t, vp, C.c_int, C.c_uint64, C.POINTER(Opts)]
    L.gz_find_blocks.argtypes = [vp, vp, C.c_size_t, vp]
    L.gz_probe_starts.argtypes = [vp, vp, vp]
    L.emu_set_sync_limit(3_000_000_000)
    store = padded(comp)
    buf = store[: len(comp)]
    b = np.asarray(bits, dtype=np.uint64)
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    h = vp()
    st = L.gz_plan_probes(C.byref(h), vp(buf.ctypes.data), buf.size, vp(b.ctypes.data), b.size, range_bytes,
                          C.byref(o))
    if st != 0:
        return st, None
    info = Info()
    L.gz_plan_info(h, C.byref(info))
    raw_ws = np.zeros(info.ws_bytes + 512, dtype=np.uint8)
    off = (-raw_ws.ctypes.data) % 256
    ws = raw_ws[off:off + info.ws_bytes]
    assert L.gz_find_blocks(h, vp(ws.ctypes.data), ws.size, None) == 0
    starts = np.zeros(b.size, dtype=np.uint64)
    rej = np.zeros(b.size, dtype=np.uint32)
    assert L.gz_probe_starts(h, vp(starts.ctypes.data), vp(rej.ctypes.data)) == 0
    L.gz_plan_destroy(h)
    return starts, rej


def stream_at(comp: bytes, bit: int, marker: int, segment_bytes: int, window: int, **opts):
    """gz_stream_open_at from `bit` to the end; returns (segment dicts, output bytes,
    gz_count_byte counts of the marker per window)."""
    L = stream_lib()
    vp = C.c_void_p
    L.gz_stream_open_at.argtypes = [C.POINTER(vp), vp, C.c_size_t, C.c_uint64, C.c_uint32, C.c_uint64,
                                    C.POINTER(Opts)]
    L.gz_count_byte.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, vp, C.c_uint64, vp]
    L.emu_set_sync_limit(3_000_000_000)
    store = padded(comp)
    buf = store[: len(comp)]
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    h = vp()
    st = L.gz_stream_open_at(C.byref(h), vp(buf.ctypes.data), buf.size, bit, marker, segment_bytes, C.byref(o))
    if st != 0:
        return st, None, None
    counts = np.zeros(1 << 14, dtype=np.uint64)
    segs, data = [], b""
    try:
        while True:
            info = StreamInfo()
            assert L.gz_stream_get_info(h, C.byref(info)) == 0
            raw_ws = np.zeros(info.ws_bytes + 512, dtype=np.uint8)
            off = (-raw_ws.ctypes.data) % 256
            ws = raw_ws[off:off + info.ws_bytes]
            out = np.zeros(max(1, info.out_bytes), dtype=np.uint8)
            assert L.gz_stream_next(h, vp(out.ctypes.data), out.size, vp(ws.ctypes.data), ws.size, None) == 0
            r = SegmentResult()
            assert L.gz_stream_wait(h, C.byref(r)) == 0
            d = {k: getattr(r, k) for k, _ in r._fields_}
            segs.append(d)
            if r.status != 0:
                break
            assert L.gz_count_byte(vp(out.ctypes.data), r.out_len, marker, len(data), window,
                                   vp(counts.ctypes.data), counts.size, None) == 0
            data += out[: r.out_len].tobytes()
            if r.done:
                break
    finally:
        L.gz_stream_destroy(h)
    return segs, data, counts[: (len(data) + window - 1) // window].astype(np.int64)


def bgzf_run(comp: bytes, **opts):
    """gz_plan_bgzf + gz_decompress_batch: (status of the plan call, output
    bytes, per-member statuses)."""
    L = lib()
    vp = C.c_void_p
    L.gz_plan_bgzf.argtypes = [C.POINTER(vp), vp, vp, C.c_size_t, vp, C.c_size_t, C.POINTER(Opts),
                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]
    L.gz_decompress_batch.argtypes = [vp, vp, C.c_size_t, vp]
    L.emu_set_sync_limit(3_000_000_000)
    store = padded(comp)
    buf = store[: len(comp)]
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    n_out, n_mem = C.c_uint64(), C.c_uint32()
    h = vp()
    st = L.gz_plan_bgzf(C.byref(h), vp(buf.ctypes.data), None, buf.size, None, 0, C.byref(o), C.byref(n_out),
                        C.byref(n_mem))
    if st != 0:
        return st, None, None
    L.gz_plan_destroy(h)
    out = np.zeros(max(1, n_out.value), dtype=np.uint8)
    st = L.gz_plan_bgzf(C.byref(h), vp(buf.ctypes.data), None, buf.size, vp(out.ctypes.data), out.size, C.byref(o),
                        C.byref(n_out), C.byref(n_mem))
    assert st == 0, st
    info = Info()
    L.gz_plan_info(h, C.byref(info))
    raw_ws = np.zeros(info.ws_bytes + 512, dtype=np.uint8)
    off = (-raw_ws.ctypes.data) % 256
    ws = raw_ws[off:off + info.ws_bytes]
    assert L.gz_decompress_batch(h, vp(ws.ctypes.data), ws.size, None) == 0
    sts = []
    for f in range(n_mem.value):
        r = Result()
        L.gz_result_get(h, f, C.byref(r))
        sts.append(r.status)
    L.gz_plan_destroy(h)
    return 0, out[: n_out.value].tobytes(), sts


def dna_run(buf, marker=0, min_len=1, bounds=None, threshold=1, max_seqs=None):
    """gz_extract_dna on the CPU executor: (list of (start, len, undetermined),
    total, per-range stats or None)."""
    L = lib()
    vp = C.c_void_p
    L.gz_extract_dna_ws.argtypes = [C.c_uint64]
    L.gz_extract_dna_ws.restype = C.c_uint64
    L.gz_extract_dna.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, vp, C.c_uint64, vp, vp,
                                 C.c_uint32, C.c_uint32, vp, vp, C.c_size_t, vp]
    L.emu_set_sync_limit(0)
    a = np.ascontiguousarray(buf)
    elem = a.dtype.itemsize
    n = a.size
    if max_seqs is None:
        max_seqs = (n + 2) // 3
    seqs = np.zeros(max(1, max_seqs), dtype=[("start", "<u8"), ("len", "<u4"), ("nu", "<u4")])
    total = np.zeros(1, dtype=np.uint64)
    nr = 0
    b = st = None
    if bounds is not None:
        b = np.asarray(bounds, dtype=np.uint64)
        nr = b.size - 1
        st = np.full(max(1, 3 * nr), 7, dtype=np.uint32)
    wsb = int(L.gz_extract_dna_ws(n))
    raw_ws = np.full(wsb + 512, 0xA5, dtype=np.uint8)
    off = (-raw_ws.ctypes.data) % 256
    ws = raw_ws[off:off + wsb]
    p = lambda x: vp(x.ctypes.data) if x is not None else None  # noqa: E731
    r = L.gz_extract_dna(vp(a.ctypes.data) if n else None, n, elem, marker, min_len, p(seqs), max_seqs, p(total),
                         p(b), nr, threshold, p(st), p(ws), wsb, None)
    assert r == 0, r
    k = min(int(total[0]), max_seqs)
    out = [(int(s["start"]), int(s["len"]), int(s["nu"])) for s in seqs[:k]]
    return out, int(total[0]), (st[: 3 * nr].reshape(nr, 3).astype(np.int64) if st is not None else None)


def members_run(comp: bytes, out_cap: int, ws_extra: int = 0, **opts):
    """gz_decompress_members on the CPU executor: (status, bytes, members)."""
    L = lib()
    vp = C.c_void_p
    L.gz_decompress_members.argtypes = [vp, C.c_size_t, vp, C.c_size_t, vp, C.c_size_t, C.POINTER(Opts), vp,
                                        C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]
    L.emu_set_sync_limit(3_000_000_000)
    store = padded(comp)
    buf = store[: len(comp)]
    o = Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    need, n_out, n_mem = C.c_uint64(), C.c_uint64(), C.c_uint32()
    st = L.gz_decompress_members(vp(buf.ctypes.data), buf.size, None, 0, None, 0, C.byref(o), None, None, None,
                                 C.byref(need))
    if st != 0:
        return st, b"", 0
    wsb = need.value + ws_extra
    raw_ws = np.zeros(wsb + 512, dtype=np.uint8)
    ws = raw_ws[(-raw_ws.ctypes.data) % 256:][:wsb]
    out = np.zeros(max(1, out_cap), dtype=np.uint8)
    st = L.gz_decompress_members(vp(buf.ctypes.data), buf.size, vp(out.ctypes.data), out_cap, vp(ws.ctypes.data),
                                 wsb, C.byref(o), None, C.byref(n_out), C.byref(n_mem), C.byref(need))
    return st, out[: n_out.value].tobytes(), n_mem.value
