"""CPU oracle for two-pass parallel gzip decompression (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers; the product path never
imports this package.  The C source (``oracle.c``) is a plain sequential
decoder written from RFC 1951/1952 plus the paper's two-pass method
(Section VI-C) and block-start checks (Section VI-A, Appendix A); it shares
no code with the device path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_HEADER, E_UNSUPPORTED, E_DATA, E_CRC, E_SIZE, E_MEM = 0, -2, -3, -4, -6, -7, -8

REASONS = {
    0: "OK", 1: "TRUNC", 2: "BTYPE3", 3: "NLEN", 4: "HLIT", 5: "HDIST", 6: "CL_OVERSUB",
    7: "CL_INCOMPLETE", 8: "REPEAT_NO_PREV", 9: "REPEAT_OVERRUN", 10: "NO_EOB", 11: "LIT_OVERSUB",
    12: "LIT_INCOMPLETE", 13: "DIST_OVERSUB", 14: "DIST_INCOMPLETE", 15: "BAD_CODE", 16: "BAD_LITLEN",
    17: "BAD_DIST", 18: "NO_DIST", 19: "TOO_FAR", 20: "MAGIC", 21: "CM", 22: "FLG", 23: "HCRC",
    24: "CRC", 25: "ISIZE", 26: "GARBAGE", 27: "NOT_ASCII", 28: "SIZE", 29: "NOT_DYNAMIC", 30: "FINAL",
}


def build(force: bool = True) -> str:
    """Compile the oracle into a shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Block(C.Structure):
    _fields_ = [("bit", C.c_int64), ("btype", C.c_int32), ("bfinal", C.c_int32),
                ("out_off", C.c_int64), ("out_len", C.c_int64), ("nsym", C.c_int64),
                ("member", C.c_int32), ("pad", C.c_int32)]


class _Gunzip(C.Structure):
    _fields_ = [("status", C.c_int), ("reason", C.c_int), ("out", C.POINTER(C.c_uint8)),
                ("out_len", C.c_size_t), ("parent", C.POINTER(C.c_int64)),
                ("blocks", C.POINTER(Block)), ("n_blocks", C.c_size_t), ("n_members", C.c_int),
                ("payload_start", C.c_size_t), ("end_bit", C.c_int64), ("trailer_at", C.c_size_t),
                ("crc_trailer", C.c_uint32), ("isize_trailer", C.c_uint32), ("crc_computed", C.c_uint32)]


class _Sym(C.Structure):
    _fields_ = [("status", C.c_int), ("reason", C.c_int), ("sym", C.POINTER(C.c_uint16)),
                ("len", C.c_size_t), ("end_bit", C.c_int64), ("final_reached", C.c_int),
                ("n_blocks", C.c_int64), ("n_syms", C.c_int64), ("n_placeholders", C.c_int64),
                ("block_bits", C.POINTER(C.c_int64))]


class _Pugz(C.Structure):
    _fields_ = [("status", C.c_int), ("reason", C.c_int), ("n_chunks", C.c_int),
                ("nominal", C.POINTER(C.c_int64)), ("start", C.POINTER(C.c_int64)),
                ("cand", C.POINTER(C.c_int64)), ("end", C.POINTER(C.c_int64)),
                ("len", C.POINTER(C.c_int64)), ("off", C.POINTER(C.c_int64)),
                ("placeholders", C.POINTER(C.c_int64)), ("valid", C.POINTER(C.c_int64)),
                ("windows", C.POINTER(C.c_uint8)), ("n_repairs", C.c_int), ("n_equivalent", C.c_int),
                ("out", C.POINTER(C.c_uint8)), ("out_len", C.c_size_t),
                ("crc_trailer", C.c_uint32), ("isize_trailer", C.c_uint32), ("crc_computed", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        u8p = C.c_void_p
        L.orc_gunzip.restype = C.POINTER(_Gunzip)
        L.orc_gunzip.argtypes = [u8p, C.c_size_t, C.c_int]
        L.orc_gunzip_free.argtypes = [C.POINTER(_Gunzip)]
        L.orc_symbolic.restype = C.POINTER(_Sym)
        L.orc_symbolic.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int64, C.c_int]
        L.orc_sym_free.argtypes = [C.POINTER(_Sym)]
        L.orc_pugz.restype = C.POINTER(_Pugz)
        L.orc_pugz.argtypes = [u8p, C.c_size_t, C.c_int]
        L.orc_pugz_mode.restype = C.POINTER(_Pugz)
        L.orc_pugz_mode.argtypes = [u8p, C.c_size_t, C.c_int, C.c_int]
        L.orc_pugz_types.restype = C.POINTER(_Pugz)
        L.orc_pugz_types.argtypes = [u8p, C.c_size_t, C.c_int, C.c_int, C.c_int]
        L.orc_block_static_types.restype = C.c_int
        L.orc_block_static_types.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int, C.POINTER(C.c_int)]
        L.orc_block_predicate_types.restype = C.c_int
        L.orc_block_predicate_types.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.orc_find_start_types.restype = C.c_int64
        L.orc_find_start_types.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int]
        L.orc_pugz_free.argtypes = [C.POINTER(_Pugz)]
        L.orc_crc32.restype = C.c_uint32
        L.orc_crc32.argtypes = [C.c_uint32, u8p, C.c_size_t]
        L.orc_block_static.restype = C.c_int
        L.orc_block_static.argtypes = [u8p, C.c_size_t, C.c_int64, C.POINTER(C.c_int)]
        L.orc_block_predicate.restype = C.c_int
        L.orc_block_predicate.argtypes = [u8p, C.c_size_t, C.c_int64, C.POINTER(C.c_int)]
        L.orc_find_start.restype = C.c_int64
        L.orc_find_start.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int64, C.c_int]
        L.orc_block_predicate_mode.restype = C.c_int
        L.orc_block_predicate_mode.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int, C.POINTER(C.c_int)]
        L.orc_find_start_mode.restype = C.c_int64
        L.orc_find_start_mode.argtypes = [u8p, C.c_size_t, C.c_int64, C.c_int64, C.c_int, C.c_int]
        L.orc_parse_header.restype = C.c_int
        L.orc_parse_header.argtypes = [u8p, C.c_size_t, C.POINTER(C.c_size_t), C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _buf(data):
    if isinstance(data, np.ndarray):
        a = np.ascontiguousarray(data, dtype=np.uint8)
    else:
        a = np.frombuffer(bytes(data), dtype=np.uint8)
    return a, a.ctypes.data_as(C.c_void_p), a.size


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def crc32(data, crc: int = 0) -> int:
    a, p, n = _buf(data)
    return int(lib().orc_crc32(crc, p, n))


def parse_header(data):
    a, p, n = _buf(data)
    h = C.c_size_t(0)
    r = C.c_int(0)
    st = lib().orc_parse_header(p, n, C.byref(h), C.byref(r))
    return st, int(h.value), REASONS.get(r.value, r.value)


class GunzipResult:
    pass


def gunzip(data, parent: bool = False) -> GunzipResult:
    """Sequential gunzip of all members; returns output, block map, trailer checks."""
    a, p, n = _buf(data)
    L = lib()
    rp = L.orc_gunzip(p, n, 1 if parent else 0)
    r = rp.contents
    out = GunzipResult()
    out.status = r.status
    out.reason = REASONS.get(r.reason, r.reason)
    out.out = _arr(r.out, r.out_len, np.uint8)
    out.parent = _arr(r.parent, r.out_len, np.int64) if parent else None
    nb = r.n_blocks
    if nb:
        blk = np.ctypeslib.as_array(C.cast(r.blocks, C.POINTER(C.c_int64)), shape=(nb * 6,)).reshape(nb, 6).copy()
        out.block_bit = blk[:, 0]
        bt = blk[:, 1].astype(np.uint64)
        out.block_type = (bt & 0xFFFFFFFF).astype(np.int32)
        out.block_final = (bt >> 32).astype(np.int32)
        out.block_out_off = blk[:, 2]
        out.block_out_len = blk[:, 3]
        out.block_nsym = blk[:, 4]
        out.block_member = (blk[:, 5].astype(np.uint64) & 0xFFFFFFFF).astype(np.int32)
    else:
        for k in ("block_bit", "block_out_off", "block_out_len", "block_nsym"):
            setattr(out, k, np.zeros(0, np.int64))
        out.block_type = out.block_final = out.block_member = np.zeros(0, np.int32)
    out.n_members = r.n_members
    out.payload_start = r.payload_start
    out.end_bit = r.end_bit
    out.trailer_at = r.trailer_at
    out.crc_trailer = r.crc_trailer
    out.isize_trailer = r.isize_trailer
    out.crc_computed = r.crc_computed
    L.orc_gunzip_free(rp)
    return out


class SymResult:
    pass


def symbolic(data, start_bit: int, stop_bit: int, first: bool) -> SymResult:
    """decompress(C_i, w_hat_i): uint16 symbols, placeholders 0x8000|j."""
    a, p, n = _buf(data)
    L = lib()
    rp = L.orc_symbolic(p, n, start_bit, stop_bit, 1 if first else 0)
    r = rp.contents
    o = SymResult()
    o.status = r.status
    o.reason = REASONS.get(r.reason, r.reason)
    o.sym = _arr(r.sym, r.len, np.uint16)
    o.end_bit = r.end_bit
    o.final_reached = bool(r.final_reached)
    o.n_blocks = r.n_blocks
    o.n_syms = r.n_syms
    o.n_placeholders = r.n_placeholders
    o.block_bits = _arr(r.block_bits, r.n_blocks, np.int64)
    L.orc_sym_free(rp)
    return o


START_DYNAMIC, START_STORED, START_FIXED = 1, 2, 4  # block types accepted as chunk starts


def block_static(data, bit: int, types: int = START_DYNAMIC):
    a, p, n = _buf(data)
    r = C.c_int(0)
    ok = lib().orc_block_static_types(p, n, bit, types, C.byref(r))
    return bool(ok), REASONS.get(r.value, r.value)


def block_predicate(data, bit: int, binary: bool = False, types: int = START_DYNAMIC):
    """Appendix A's checks at one bit (binary: without the ASCII test; types:
    the block types accepted as starts)."""
    a, p, n = _buf(data)
    r = C.c_int(0)
    ok = lib().orc_block_predicate_types(p, n, bit, 0 if binary else 1, types, C.byref(r))
    return bool(ok), REASONS.get(r.value, r.value)


def find_start(data, lo_bit: int, hi_bit: int, static_only: bool = False, binary: bool = False,
               types: int = START_DYNAMIC) -> int:
    a, p, n = _buf(data)
    return int(lib().orc_find_start_types(p, n, lo_bit, hi_bit, 1 if static_only else 0, 0 if binary else 1,
                                          types))


class PugzResult:
    pass


def pugz(data, n_chunks: int, binary: bool = False, types: int = START_DYNAMIC) -> PugzResult:
    """The two-pass method on the CPU: per-chunk starts, ends, lengths, windows,
    output (binary: block starts searched without the ASCII test; types: the
    block types accepted as chunk starts)."""
    a, p, n = _buf(data)
    L = lib()
    rp = L.orc_pugz_types(p, n, n_chunks, 0 if binary else 1, types)
    r = rp.contents
    o = PugzResult()
    o.status = r.status
    o.reason = REASONS.get(r.reason, r.reason)
    N = r.n_chunks
    o.n_chunks = N
    o.nominal = _arr(r.nominal, N + 1, np.int64)
    for k in ("start", "cand", "end", "len", "off", "placeholders", "valid"):
        setattr(o, k, _arr(getattr(r, k), N, np.int64))
    o.windows = _arr(r.windows, N * 32768, np.uint8).reshape(N, 32768) if N else None
    o.n_repairs = r.n_repairs
    o.n_equivalent = r.n_equivalent
    o.out = _arr(r.out, r.out_len, np.uint8)
    o.crc_trailer = r.crc_trailer
    o.isize_trailer = r.isize_trailer
    o.crc_computed = r.crc_computed
    L.orc_pugz_free(rp)
    return o
