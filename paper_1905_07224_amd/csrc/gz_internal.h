// Internal layout shared by the host planner and the device passes.
#pragma once
#include <stdint.h>

namespace gzgpu {

constexpr uint64_t NONE = ~0ull;
constexpr uint32_t WINDOW = 32768;       // DEFLATE history (RFC 1951 section 2; paper Section III)
constexpr uint32_t FLUSH_UNIT = 512;     // symbols moved from LDS to HBM at a time
constexpr uint32_t TRANSLATE_TILE = 8192;
constexpr uint32_t SYM_SLACK = 2048;     // symbols added to every chunk's capacity
constexpr uint32_t DEFAULT_RING = 512;   // symbols of LDS history per decoding wave
constexpr uint64_t DEFAULT_CHUNK_BYTES = 40 << 10;  // nominal compressed bytes per chunk
constexpr uint64_t SCRATCH_BYTES = 256ull << 20;    // static workspace of gz_decompress_static, per GPU
// LDS bytes of one decoding wave (tables + a ring of `win` 16-bit symbols), upper bound
constexpr uint32_t inflate_lds_bytes(uint32_t win) { return 7424u + 2u * win; }

// chunk flags
enum : uint32_t {
  CF_FIRST = 1u,        // first chunk of its file: starts at the payload, empty context
  CF_CARRIED = 2u,      // (with CF_FIRST) a segment's first chunk: its context is the carried window
};

// Compressed bytes past a segment's stop that its last chunk may still decode
// (the rest of the block that holds the stop).  The symbol capacity of that
// chunk counts them; a longer block reports a capacity error.
constexpr uint64_t STOP_MARGIN_BYTES = 128 << 10;

// chunk state flags
enum : uint32_t {
  CS_FINAL = 1u,        // decoding reached the final block
  CS_EMPTY = 2u,        // no start in range (or dropped)
  CS_EXTENDED = 4u,     // continued past the first stop
  CS_REPAIRED = 8u,     // start replaced by the previous chunk's end
  CS_OVERFLOW = 16u,    // symbol capacity exceeded before the stop
  CS_UNCONFIRMED = 32u, // its deferred confirmation blocks failed (redone by k_redo)
  CS_CUT = 64u,         // pass 1 outgrew its capacity: symbols stored up to cut_bit only (continued by k_stitch)
};

// device status codes (same numbers as the public GZ_E_*)
enum : int32_t {
  ST_OK = 0,
  ST_UNSUPPORTED = -3,
  ST_DATA = -4,
  ST_CAPACITY = -5,
  ST_CRC = -6,
  ST_SIZE = -7,
};

// CRC-32 of the output (RFC 1952 section 8) on the device: units of
// CRC_UNIT bytes, CRC_LANE bytes per lane.  Constants set by the host, in the
// reflected representation (x^0 = 0x80000000): xpow[k] = x^(8 * 2^k) mod P
// (k < CRC_XPOW), then lanepow[m] = x^(8 * CRC_LANE * m) mod P (m < 64).
constexpr uint32_t CRC_UNIT = 65536;
constexpr uint32_t CRC_LANE = CRC_UNIT / 64;
constexpr int CRC_XPOW = 48;
constexpr int CRC_CONSTS = CRC_XPOW + 64;
constexpr uint32_t CRC_POLY = 0xEDB88320u;

struct FileDesc {
  const uint8_t *comp;     // device address of the .gz bytes
  uint64_t comp_len;
  uint64_t payload_bit;    // 8 * payload start byte
  uint64_t trailer_byte;   // comp_len - 8
  uint8_t *out;
  uint64_t out_cap;
  uint32_t first_chunk;
  uint32_t n_chunks;
  uint32_t isize;
  uint32_t crc;
  uint64_t pool_base;      // this file's part of the symbol pool (elements)
  uint64_t pool_elems;
  uint64_t crc_unit0;      // first CRC unit of this file (units of all earlier files' out_cap)
  // a segment of a longer member (bounded-memory streaming): decoding starts
  // at payload_bit, a proven block boundary, and the last chunk stops at the
  // first block header at or past stop_bit; NONE: decode to the final block
  uint64_t stop_bit;
  uint64_t out_before;     // bytes of the member before this segment (ISIZE is checked on the sum)
  uint32_t crc_in;         // CRC-32 of those bytes (0 for none)
  uint32_t win_valid;      // real bytes in the carried window (the first chunk's window slot), 0: none
  uint32_t mode;           // FD_* below
  uint32_t pad2;
};

// file modes
enum : uint32_t {
  FD_PROBE = 1u,    // block-start probe: one chunk, decodes its first block (plus the confirmation)
  FD_NOCHECK = 2u,  // decoding began inside the member: the trailer's CRC-32 and ISIZE do not apply
  FD_MEMBERS = 4u,  // more members may follow: the trailer is the 8 bytes after the final block
  FD_BINARY = 8u,   // binary input: block-start checks without the ASCII test of the literals
  FD_STORED_STARTS = 16u,  // stored blocks are chunk-start candidates too
};

struct ChunkDesc {
  uint64_t lo_bit;         // candidate range [lo_bit, hi_bit), bits from the file start
  uint64_t hi_bit;
  uint64_t sym_off;        // element offset of the chunk's symbols in the pool (set on the device)
  uint64_t sym_cap;        // capacity in symbols, multiple of FLUSH_UNIT (set on the device)
  uint32_t file;
  uint32_t index;          // chunk index within its file
  uint32_t flags;
  uint32_t pad;
};

struct ChunkState {
  uint64_t cand;           // smallest start passing the static checks (scan), NONE if none
  uint64_t start;          // accepted start bit, NONE if the chunk is empty
  uint64_t found;          // start the block-start checks accepted, before any repair (NONE: none)
  uint64_t end;            // bit where decoding stopped (a block start, or the end of the final block)
  uint64_t len;            // symbols produced up to the stop
  uint64_t out_off;        // output offset
  uint64_t needed;         // symbols produced when the capacity overflowed
  uint64_t n_syms;
  uint64_t n_placeholders;
  int32_t status;
  uint32_t flags;
  uint32_t n_blocks;
  uint32_t retries;
  uint32_t valid;          // real history bytes before the chunk, capped at 32768
  uint32_t pad;            // confirmation blocks owed past the stop (deferred), else 0
  // block-start search statistics (Appendix A's stages), counted where the
  // search ran (it ends at the first candidate that passes)
  uint32_t stage1;         // candidates past the cheap header checks, given the full table check
  uint32_t stage2;         // of those, candidates whose code tables are valid
  uint32_t trial_rej;      // candidates whose trial block failed (ASCII, size, decoding)
  uint32_t confirm_rej;    // candidates whose five confirmation blocks failed
  // CS_CUT: pass 1 outgrew the capacity and stored only the symbols before
  // cut_bit (a block boundary; len of them, cut_blocks blocks); the stitch
  // pass continues from there
  uint64_t cut_bit;
  uint32_t cut_blocks;
  uint32_t pad2;
};

// A chunk with an accepted start, in chunk order (window propagation walks these).
struct AccEntry {
  uint64_t sym_off;
  uint64_t len;            // |D_j|
  uint32_t chunk;
  uint32_t pad;            // bit 0: the first chunk of its file; bit 1: its window is carried in
};

struct FileState {
  uint64_t out_len;
  uint64_t out_needed;
  uint64_t n_syms;
  uint64_t n_placeholders;
  uint64_t n_blocks;
  int32_t status;
  uint32_t n_repairs;
  uint32_t n_extended;
  uint32_t n_nonempty;
  uint32_t n_retries;
  uint32_t overflow;
  uint32_t size_bad;       // length differs from ISIZE (reported after the CRC, as RFC 1952 checks it first)
  uint32_t crc_acc;        // XOR of the units' shifted raw CRCs
  uint32_t crc_out;        // CRC-32 of the output (with the bytes before the segment)
  uint32_t is_final;       // the member's final block was decoded (the trailer is checked)
  uint64_t end_bit;        // where the last accepted chunk stopped
  uint32_t trailer_crc;    // the member's trailer: CRC-32 and ISIZE
  uint32_t trailer_isize;
};

struct Counters {
  uint32_t inflate_next;   // persistent work queue head
  uint32_t stitch_next;
  uint32_t translate_next;
  uint32_t confirm_next;
  uint32_t redo_next;
  uint32_t pad[11];
};

// Workspace: offsets from the workspace base (all 256-byte aligned).
struct Layout {
  uint64_t files_off;      // FileDesc[F]
  uint64_t chunks_off;     // ChunkDesc[N]
  uint64_t order_off;      // uint32[N]: inflate work order
  uint64_t crc_off;        // uint32[CRC_XPOW] powers of x for the CRC combine (in the uploaded table)
  uint64_t table_bytes;    // bytes uploaded from the host (files + chunks + order + scan list + crc)
  uint64_t cstate_off;     // ChunkState[N]
  uint64_t fstate_off;     // FileState[F]
  uint64_t counters_off;   // Counters
  uint64_t tiles_off;      // uint64[N+1] translate tile prefix
  uint64_t acc_off;        // uint32[N+1] accepted chunks before chunk j, then AccEntry[N] in chunk order
  uint64_t maps_off;       // uint16[2][S][32768] propagation segment maps and their prefix compositions, S = ceil(N / 64)
  uint64_t segwin_off;     // uint8[S][32768] input window of each propagation segment
  uint64_t win_off;        // uint8[N][32768] resolved windows
  uint64_t carry_off;      // uint8[32768] the window after the last chunk (bounded-memory streaming)
  uint64_t sym_off;        // uint16 symbol pool
  uint64_t sym_elems;
  uint64_t total;
};

}  // namespace gzgpu
