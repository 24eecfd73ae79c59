// HIP kernels of the two-pass gzip path (gfx950).
//
//   k_init       clear per-chunk and per-file state (a kernel, so the whole
//                sequence can be captured in a graph)
//   k_scan       block-start search (Section VI-A, Appendix A): one lane per
//                candidate bit, survivors checked by the whole wave
//   k_inflate    pass 1, decompress(C_i, w_hat_i) (Section VI-C): one wave per
//                chunk from a persistent work queue, tables and the recent
//                history in LDS, 16-bit symbols to HBM
//   k_stitch     chunks whose stop was not the next accepted start continue
//   k_finalize   stitch check, sequential repair when a start is off the
//                block chain, output offsets (exclusive scan of |D_i|)
//   k_propagate  pass 2a: windows resolved chunk after chunk
//   k_translate  pass 2b: every U_j replaced by w_i[j], written to the output
#include <hip/hip_runtime.h>

#include "gz_device.h"
#include "gz_internal.h"

namespace gzgpu {

// ---------------------------------------------------------------------------
// Inflater: one wave decodes blocks of one chunk.
// ---------------------------------------------------------------------------

template <int WIN>
struct InflateLDS {
  TablesLDS t;
  alignas(16) uint16_t ring[WIN];  // the last WIN symbols produced, by position mod WIN
};

struct DecodeResult {
  int status;        // D_OK or failure
  bool confirmed;    // the check blocks all passed (or none were asked)
  bool final_seen;
  uint64_t end;      // stop bit
  uint64_t len;      // symbols up to the stop
  uint32_t blocks;
};

template <int WIN>
struct Inflater {
  // The ring holds the whole DEFLATE window (32768 symbols), so every match
  // source is in LDS: a source pos - d + k (d <= 32768) is read before any
  // write of this match reaches its slot, and the unit being moved to HBM is
  // never older than 512 + 258 symbols.
  static_assert(WIN == 32768, "the LDS history must hold the whole window");
  static constexpr uint32_t RMASK = WIN - 1;

  InflateLDS<WIN> &sh;
  WaveBits br;
  uint16_t *D;       // chunk symbols in HBM
  uint64_t cap;      // symbol capacity
  uint64_t pos;      // symbols produced
  uint64_t flushed;  // symbols stored to HBM (multiple of FLUSH_UNIT)
  uint64_t nsyms;
  uint32_t nph;      // per lane placeholder count
  uint32_t nph_stop; // per lane placeholder count at the stop (symbols of D_i only)
  bool first;        // empty context
  bool over;         // capacity exceeded somewhere

  __device__ Inflater(InflateLDS<WIN> &s) : sh(s) {}

  __device__ __forceinline__ void flush_unit() {
    wave_sync();
    const int lane = lane_id();
    const uint64_t u = flushed;
    const uint4 v = *reinterpret_cast<const uint4 *>(&sh.ring[(u + 8u * lane) & RMASK]);
    if (u + FLUSH_UNIT <= cap) {
      *reinterpret_cast<uint4 *>(D + u + 8u * lane) = v;
    } else {
      over = true;
    }
    flushed = u + FLUSH_UNIT;
  }
  __device__ __forceinline__ void maybe_flush() {
    while (pos > flushed && pos - flushed >= FLUSH_UNIT) flush_unit();
  }
  __device__ void flush_all() {
    while (flushed < pos) flush_unit();
  }

  __device__ __forceinline__ void put_lit(uint32_t c) {
    if (lane_id() == 0) sh.ring[pos & RMASK] = (uint16_t)c;
    pos++;
    if (pos - flushed >= FLUSH_UNIT) flush_unit();
  }

  // Copy len symbols from d back.  The source of element k is before the
  // match start: pos - d + k when d >= 64 (an earlier 64-step already wrote
  // it), pos - d + (k mod d) when d < 64.  Sources before the chunk are the
  // placeholders U_j.
  __device__ __forceinline__ int put_match(uint32_t len, uint32_t d) {
    if (first && (uint64_t)d > pos) return D_FAR;
    const int lane = lane_id();
    if (d >= 64u) {
      for (uint32_t k0 = 0; k0 < len; k0 += 64) {
        wave_sync();
        const uint32_t k = k0 + (uint32_t)lane;
        if (k < len) {
          const int64_t src = (int64_t)pos + k - d;
          const uint32_t v = src < 0 ? 0x8000u | (uint32_t)(32768 + src) : (uint32_t)sh.ring[src & RMASK];
          nph += v >> 15;
          sh.ring[(pos + k) & RMASK] = (uint16_t)v;
        }
      }
    } else {
      const float rd = 1.0f / (float)d;
      for (uint32_t k0 = 0; k0 < len; k0 += 64) {
        wave_sync();
        const uint32_t k = k0 + (uint32_t)lane;
        if (k < len) {
          int q = (int)((float)k * rd);
          int r = (int)k - q * (int)d;
          if (r >= (int)d) r -= (int)d;
          if (r < 0) r += (int)d;
          const int64_t src = (int64_t)pos - d + r;
          const uint32_t v = src < 0 ? 0x8000u | (uint32_t)(32768 + src) : (uint32_t)sh.ring[src & RMASK];
          nph += v >> 15;
          sh.ring[(pos + k) & RMASK] = (uint16_t)v;
        }
      }
    }
    pos += len;
    maybe_flush();
    return D_OK;
  }

  // Stored block: LEN raw bytes copied 64 at a time.
  __device__ int stored(bool check) {
    const int lane = lane_id();
    br.pos = (br.pos + 7) & ~7ull;
    uint64_t v = br.next();
    uint32_t n = (uint32_t)(v & 0xFFFFu), nn = (uint32_t)((v >> 16) & 0xFFFFu);
    br.skip(32);
    if (br.past_end()) return D_TRUNC;
    if ((n ^ 0xFFFFu) != nn) return D_BAD;
    const uint64_t fb = br.pos >> 3;
    if (br.pos + 8ull * n > br.s.end_bits) return D_TRUNC;
    for (uint32_t k0 = 0; k0 < n; k0 += 64) {
      const uint32_t k = k0 + (uint32_t)lane;
      bool bad = false;
      if (k < n) {
        uint32_t c = br.s.byte(fb + k);
        bad = check && !ascii_text(c);
        sh.ring[(pos + (uint32_t)lane) & RMASK] = (uint16_t)c;
      }
      if (__ballot(bad)) return D_ASCII;
      pos += min(64u, n - k0);
      maybe_flush();
    }
    br.pos += 8ull * n;
    return D_OK;
  }

  // Huffman-coded block body until end-of-block (section 3.2.5).
  __device__ int huffman(bool check, bool no_dist, uint64_t size_cap, uint64_t blk0) {
    // each symbol consumes at least one bit: the remaining bits bound the loop
    const uint64_t budget = br.s.end_bits - br.pos + 1;
    for (uint64_t it = 0;; it++) {
      if (it > budget) return D_BAD;
      const uint64_t v = br.next();
      uint32_t e = uni32(sh.t.lit[v & ((1u << LIT_BITS) - 1)]);
      uint32_t kind = (e >> 4) & 15u;
      if (kind == K_LONG) {
        e = decode_long<LIT_BITS, TREE_LIT>(v, &sh.t.li, sh.t.lsorted);
        kind = (e >> 4) & 15u;
      }
      const uint32_t cl = e & 15u;
      nsyms++;
      if (kind == K_LIT) {
        const uint32_t c = (e >> 8) & 255u;
        if (check && !ascii_text(c)) return D_ASCII;
        put_lit(c);
        br.skip(cl);
        if (br.past_end()) return D_TRUNC;
        continue;
      }
      if (kind == K_EOB) {
        br.skip(cl);
        return br.past_end() ? D_TRUNC : D_OK;
      }
      if (kind != K_LEN) return D_BAD;
      const uint32_t ex = (e >> 8) & 255u;
      const uint32_t len = (e >> 16) + ((uint32_t)(v >> cl) & ((1u << ex) - 1u));
      uint32_t used = cl + ex;
      if (no_dist) return D_BAD;
      const uint64_t v2 = v >> used;
      uint32_t ed = uni32(sh.t.dist[v2 & ((1u << DIST_BITS) - 1)]);
      uint32_t kd = (ed >> 4) & 15u;
      if (kd == K_LONG) {
        ed = decode_long<DIST_BITS, TREE_DIST>(v2, &sh.t.di, sh.t.dsorted);
        kd = (ed >> 4) & 15u;
      }
      if (kd != K_LEN) return D_BAD;
      const uint32_t dl = ed & 15u, dex = (ed >> 8) & 255u;
      const uint32_t dist = (ed >> 16) + ((uint32_t)(v2 >> dl) & ((1u << dex) - 1u));
      used += dl + dex;
      br.skip(used);
      if (br.past_end()) return D_TRUNC;
      int r = put_match(len, dist);
      if (r) return r;
      if (pos - blk0 >= size_cap) return D_SIZE;
    }
  }

  // One block.  check: ASCII literals (block-start confirmation); strict: the
  // candidate block itself (must be a non-final dynamic block with a complete
  // literal/length code and a size in (1 KiB, 4 MiB)).
  __device__ int block(bool check, bool strict, bool *final_out) {
    const uint64_t v = br.next();
    const uint32_t bfinal = (uint32_t)(v & 1u), btype = (uint32_t)((v >> 1) & 3u);
    br.skip(3);
    if (br.past_end()) return D_TRUNC;
    *final_out = bfinal != 0;
    if (strict && (bfinal || btype != 2u)) return D_STATIC;
    const uint64_t blk0 = pos;
    int r;
    if (btype == 0u) {
      r = stored(check);
    } else if (btype == 1u) {
      fixed_tables(sh.t);
      r = huffman(check, false, ~0ull, blk0);
    } else if (btype == 2u) {
      bool nd = false;
      r = read_dynamic_tables(br, sh.t, strict, true, &nd);
      if (r == D_OK) r = huffman(check, nd, strict ? (4ull << 20) : ~0ull, blk0);
    } else {
      r = D_BAD;
    }
    if (r == D_OK && strict && !(pos - blk0 > 1024u && pos - blk0 < (4ull << 20))) r = D_SIZE;
    return r;
  }

  // Decode whole blocks from bit `start`, with `pos` symbols already produced,
  // until the first block header at or past `stop` (or a final block).  The
  // first `check_blocks` blocks are the block-start trial and confirmation; if
  // the stop comes first they are still decoded, then the stop is reported.
  __device__ DecodeResult run(uint64_t start, uint64_t stop, uint32_t check_blocks) {
    DecodeResult res;
    res.status = D_OK;
    res.confirmed = check_blocks == 0;
    res.final_seen = false;
    res.end = NONE;
    res.len = 0;
    res.blocks = 0;
    br.init(start);
    uint32_t nb = 0;
    // a block header is at least 3 bits: the remaining bits bound the blocks
    const uint64_t budget = (br.s.end_bits - br.pos) / 3 + 2;
    for (uint64_t it = 0;; it++) {
      if (it > budget) {
        res.status = D_BAD;
        break;
      }
      if (res.end == NONE && br.pos >= stop) {
        res.end = br.pos;
        res.len = pos;
        nph_stop = nph;
      }
      if (res.end != NONE && nb >= check_blocks) break;
      bool fin = false;
      const bool check = nb < check_blocks;
      int r = block(check, check && nb == 0, &fin);
      if (r != D_OK) {
        res.status = r;
        break;
      }
      nb++;
      if (fin) {
        res.final_seen = res.end == NONE;
        if (res.end == NONE) {
          res.end = br.pos;
          res.len = pos;
          nph_stop = nph;
        }
        nb = check_blocks > nb ? check_blocks : nb;  // a final block ends the confirmation
        break;
      }
    }
    res.blocks = nb;
    if (res.end == NONE) nph_stop = nph;
    if (res.status == D_OK) res.confirmed = true;
    flush_all();
    return res;
  }
};

template <int WIN>
__device__ __forceinline__ void inflater_setup(Inflater<WIN> &inf, const FileDesc &fd, const ChunkDesc &cd,
                                               uint16_t *pool) {
  inf.br.s.init(fd.comp, fd.comp_len);
  inf.D = pool + cd.sym_off;
  inf.cap = cd.sym_cap;
  inf.pos = 0;
  inf.flushed = 0;
  inf.nsyms = 0;
  inf.nph = 0;
  inf.nph_stop = 0;
  inf.first = (cd.flags & CF_FIRST) != 0;
  inf.over = false;
}

// Next chunk of the same file that has a start (scan candidate or accepted).
__device__ __forceinline__ uint64_t next_start(const FileDesc &fd, const ChunkState *cs, uint32_t c, bool accepted,
                                               uint32_t *which) {
  const uint32_t endc = fd.first_chunk + fd.n_chunks;
  for (uint32_t j = c + 1; j < endc; j++) {
    uint64_t s = accepted ? cs[j].start : cs[j].cand;
    if (s != NONE) {
      if (which) *which = j;
      return s;
    }
  }
  if (which) *which = endc;
  return NONE;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Decode chunk c from scratch (pass 1 for one chunk).
template <int WIN>
__device__ void inflate_chunk(InflateLDS<WIN> &sh, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                              uint16_t *pool, uint32_t c) {
  const int lane = lane_id();
  const ChunkDesc cd = chunks[c];
  const FileDesc fd = files[cd.file];
  const bool first = (cd.flags & CF_FIRST) != 0;
  uint64_t b = first ? fd.payload_bit : uni64(cs[c].cand);
  const uint64_t stop = first || b != NONE ? uni64(next_start(fd, cs, c, false, nullptr)) : NONE;
  Inflater<WIN> inf(sh);
  uint32_t retries = 0;
  // each retry moves the candidate forward by at least one bit
  const uint64_t max_tries = cd.hi_bit - cd.lo_bit + 2;
  for (uint64_t tries = 0;; tries++) {
    if (tries > max_tries) b = NONE;
    if (b == NONE || (!first && b >= cd.hi_bit)) {
      if (lane == 0) {
        cs[c].start = NONE;
        cs[c].end = NONE;
        cs[c].len = 0;
        cs[c].flags = CS_EMPTY;
        cs[c].retries = retries;
        cs[c].status = ST_OK;
      }
      return;
    }
    inflater_setup(inf, fd, cd, pool);
    DecodeResult r = inf.run(b, stop, first ? 0u : 6u);
    if (r.status != D_OK && (first || r.blocks >= 6u)) {
      if (lane == 0) {
        cs[c].start = b;
        cs[c].end = r.end;
        cs[c].len = r.len;
        cs[c].status = ST_DATA;
        cs[c].flags = 0;
        cs[c].retries = retries;
      }
      return;
    }
    if (r.status == D_OK) {
      uint32_t ph = wave_sum(inf.nph_stop);
      bool overflow = inf.over && r.len > cd.sym_cap;
      if (lane == 0) {
        cs[c].start = b;
        cs[c].end = r.end;
        cs[c].len = r.len;
        cs[c].status = overflow ? ST_CAPACITY : ST_OK;
        cs[c].needed = overflow ? r.len : 0;
        cs[c].flags = (r.final_seen ? CS_FINAL : 0u) | (overflow ? CS_OVERFLOW : 0u);
        cs[c].n_blocks = r.blocks;
        cs[c].n_syms = inf.nsyms;
        cs[c].n_placeholders = ph;
        cs[c].retries = retries;
      }
      return;
    }
    // the candidate failed the trial decode or the confirmation: next one
    retries++;
    b = wave_find_start(inf.br.s, b + 1, cd.hi_bit, sh.t);
  }
}

// ---------------------------------------------------------------------------
// k_init
// ---------------------------------------------------------------------------

__global__ void k_init(ChunkState *cs, uint32_t n_chunks, FileState *fs, uint32_t n_files, Counters *ctr) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_chunks) {
    ChunkState z;
    z.cand = NONE;
    z.start = NONE;
    z.end = NONE;
    z.len = 0;
    z.out_off = 0;
    z.needed = 0;
    z.n_syms = 0;
    z.n_placeholders = 0;
    z.status = ST_OK;
    z.flags = 0;
    z.n_blocks = 0;
    z.retries = 0;
    z.valid = 0;
    z.pad = 0;
    cs[i] = z;
  }
  if (i < n_files) {
    FileState f = {};
    fs[i] = f;
  }
  if (i < sizeof(Counters) / 4) reinterpret_cast<uint32_t *>(ctr)[i] = 0u;
}

// ---------------------------------------------------------------------------
// k_scan: for every chunk after the first of its file, the smallest bit in
// [lo_bit, hi_bit) passing the static checks.  `groups` workgroups share one
// chunk and sweep 256-bit tiles in an interleaved order; a tile is skipped
// once a passing candidate before it is known.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_scan(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                              const uint32_t *scan_list, uint32_t n_scan, uint32_t groups) {
  __shared__ TablesLDS sh[4];
  const uint32_t item = blockIdx.x / groups, g = blockIdx.x % groups;
  if (item >= n_scan) return;
  const uint32_t c = scan_list[item];
  const ChunkDesc cd = chunks[c];
  Src s;
  s.init(files[cd.file].comp, files[cd.file].comp_len);
  const int wave = (int)uni32(threadIdx.x >> 6), lane = lane_id();
  unsigned long long *cand = (unsigned long long *)&cs[c].cand;
  for (uint64_t t = g;; t += groups) {
    const uint64_t tile = cd.lo_bit + t * 256u;
    if (tile >= cd.hi_bit) break;
    const uint64_t cur = uni64(__hip_atomic_load(cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (cur <= tile) break;
    const uint64_t b0 = tile + 64u * (uint64_t)wave;
    const uint64_t b = b0 + (uint64_t)lane;
    const bool p = b < cd.hi_bit && start_stage1(s, b);
    uint64_t m = __ballot(p);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const uint64_t bb = b0 + (uint64_t)l;
      if (bb >= uni64(__hip_atomic_load(cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) break;
      if (start_stage2(s, bb, sh[wave])) {
        if (lane == 0) atomicMin(cand, (unsigned long long)bb);
        break;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_capacity: one workgroup per file.  A chunk decodes from its start to the
// next chunk start found by the scan, so its symbol capacity is sized from
// that span: factor * span bytes + slack, rounded to the flush unit.  The
// spans partition the payload, so the file's pool of
// factor * (P + N) + N * (slack + unit) symbols always suffices.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_capacity(const FileDesc *files, ChunkDesc *chunks, const ChunkState *cs,
                                                  uint32_t factor) {
  __shared__ uint64_t part[256];
  __shared__ uint64_t nxt[256];
  const uint32_t f = blockIdx.x;
  const FileDesc fd = files[f];
  const uint32_t c0 = fd.first_chunk, n = fd.n_chunks;
  const int tid = (int)threadIdx.x;
  const uint64_t end_bit = 8ull * fd.trailer_byte;
  // pass 1, last tile first: next start after each chunk (suffix minimum)
  uint64_t later = end_bit;
  const uint32_t ntiles = (n + 255) / 256;
  for (uint32_t t = ntiles; t-- > 0;) {
    const uint32_t i = t * 256 + (uint32_t)tid;
    uint64_t s = NONE;
    if (i < n) s = (chunks[c0 + i].flags & CF_FIRST) ? fd.payload_bit : cs[c0 + i].cand;
    part[tid] = s;
    __syncthreads();
    // inclusive suffix minimum within the tile
    for (int o = 1; o < 256; o <<= 1) {
      const uint64_t b = tid + o < 256 ? part[tid + o] : NONE;
      __syncthreads();
      part[tid] = part[tid] < b ? part[tid] : b;
      __syncthreads();
    }
    const uint64_t after = tid + 1 < 256 ? part[tid + 1] : NONE;
    nxt[tid] = after < later ? after : later;
    const uint64_t tile_min = part[0];
    __syncthreads();
    if (i < n) {
      uint64_t cap = 0;
      if (s != NONE && s < end_bit) {
        const uint64_t e = nxt[tid] < end_bit ? nxt[tid] : end_bit;
        const uint64_t span = e > s ? (e - s + 7) / 8 : 1;
        cap = ((uint64_t)factor * span + SYM_SLACK + FLUSH_UNIT - 1) / FLUSH_UNIT * FLUSH_UNIT;
      }
      chunks[c0 + i].sym_cap = cap;
    }
    later = tile_min < later ? tile_min : later;
    __syncthreads();
  }
  // pass 2: exclusive prefix sum of the capacities
  uint64_t carry = fd.pool_base;
  for (uint32_t t = 0; t < ntiles; t++) {
    const uint32_t i = t * 256 + (uint32_t)tid;
    const uint64_t cap = i < n ? chunks[c0 + i].sym_cap : 0;
    part[tid] = cap;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const uint64_t a = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      __syncthreads();
    }
    if (i < n) chunks[c0 + i].sym_off = carry + part[tid] - cap;
    carry += part[255];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_inflate: persistent; each wave pops chunk indices from the work queue.
// ---------------------------------------------------------------------------

template <int WIN>
__global__ __launch_bounds__(64) void k_inflate(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                                const uint32_t *order, uint32_t n, Counters *ctr, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  for (uint32_t it = 0; it <= n; it++) {
    uint32_t item = 0;
    if (lane_id() == 0) item = atomicAdd(&ctr->inflate_next, 1u);
    item = uni(item);
    if (item >= n) break;
    inflate_chunk<WIN>(sh, files, chunks, cs, pool, order[item]);
  }
}

// Continue chunk c from its recorded end until the first block at or past `stop`.
template <int WIN>
__device__ void extend_chunk(InflateLDS<WIN> &sh, const FileDesc &fd, const ChunkDesc &cd, ChunkState *cs,
                             uint16_t *pool, uint32_t c, uint64_t stop) {
  const int lane = lane_id();
  Inflater<WIN> inf(sh);
  inflater_setup(inf, fd, cd, pool);
  const uint64_t len = uni64(cs[c].len);
  const uint64_t e = uni64(cs[c].end);
  // bring the recent history back into the ring
  const uint64_t h0 = len > (uint64_t)WIN ? len - WIN : 0;
  for (uint64_t p = h0 + (uint64_t)lane; p < len; p += 64)
    sh.ring[p & (WIN - 1)] = p < cd.sym_cap ? inf.D[p] : (uint16_t)0;
  wave_sync();
  inf.pos = len;
  inf.flushed = len & ~(uint64_t)(FLUSH_UNIT - 1);
  DecodeResult r = inf.run(e, stop, 0u);
  uint32_t ph = wave_sum(inf.nph_stop);
  if (lane == 0) {
    bool overflow = inf.over && r.len > cd.sym_cap;
    cs[c].end = r.end;
    cs[c].len = r.len;
    cs[c].n_blocks += r.blocks;
    cs[c].n_syms += inf.nsyms;
    cs[c].n_placeholders += ph;
    cs[c].flags |= CS_EXTENDED | (r.final_seen ? CS_FINAL : 0u) | (overflow ? CS_OVERFLOW : 0u);
    if (r.status != D_OK) cs[c].status = ST_DATA;
    else if (overflow) {
      cs[c].status = ST_CAPACITY;
      cs[c].needed = r.len;
    }
  }
}

// Decode chunk c again from `start` with a placeholder context (repair).
template <int WIN>
__device__ void redecode_chunk(InflateLDS<WIN> &sh, const FileDesc &fd, const ChunkDesc &cd, ChunkState *cs,
                               uint16_t *pool, uint32_t c, uint64_t start, uint64_t stop) {
  const int lane = lane_id();
  Inflater<WIN> inf(sh);
  inflater_setup(inf, fd, cd, pool);
  DecodeResult r = inf.run(start, stop, 0u);
  uint32_t ph = wave_sum(inf.nph_stop);
  if (lane == 0) {
    bool overflow = inf.over && r.len > cd.sym_cap;
    cs[c].start = start;
    cs[c].end = r.end;
    cs[c].len = r.len;
    cs[c].n_blocks = r.blocks;
    cs[c].n_syms = inf.nsyms;
    cs[c].n_placeholders = ph;
    cs[c].flags = CS_REPAIRED | (r.final_seen ? CS_FINAL : 0u) | (overflow ? CS_OVERFLOW : 0u);
    cs[c].status = r.status != D_OK ? ST_DATA : overflow ? ST_CAPACITY : ST_OK;
    cs[c].needed = overflow ? r.len : 0;
  }
}

// ---------------------------------------------------------------------------
// k_stitch: a chunk stopped at the next chunk's scan candidate; if the next
// accepted start is later (the candidate failed its trial decode, or the next
// chunks are empty), continue to it.
// ---------------------------------------------------------------------------

template <int WIN>
__global__ __launch_bounds__(64) void k_stitch(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                               uint32_t n, Counters *ctr, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  for (uint32_t it = 0; it <= n; it++) {
    uint32_t c = 0;
    if (lane_id() == 0) c = atomicAdd(&ctr->stitch_next, 1u);
    c = uni(c);
    if (c >= n) break;
    const ChunkDesc cd = chunks[c];
    const FileDesc fd = files[cd.file];
    if (uni64(cs[c].start) == NONE || uni(cs[c].status) != ST_OK || (uni(cs[c].flags) & CS_FINAL)) continue;
    const uint64_t nf = uni64(next_start(fd, cs, c, true, nullptr));
    const uint64_t e = uni64(cs[c].end);
    if (e < nf || nf == NONE) extend_chunk<WIN>(sh, fd, cd, cs, pool, c, nf);
  }
}

// ---------------------------------------------------------------------------
// k_finalize: one workgroup per file.  Checks that every accepted start is
// the previous chunk's end, repairs sequentially if not, then the exclusive
// scan of the chunk lengths gives the output offsets.
// ---------------------------------------------------------------------------

template <int WIN>
__global__ __launch_bounds__(256) void k_finalize(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                                  FileState *fs, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  __shared__ int bad;
  __shared__ uint64_t part[256];
  const uint32_t f = blockIdx.x;
  const FileDesc fd = files[f];
  const uint32_t c0 = fd.first_chunk, c1 = fd.first_chunk + fd.n_chunks;
  const int tid = (int)threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  // parallel check of the chain
  for (uint32_t j = c0 + tid; j < c1; j += blockDim.x) {
    const ChunkState sj = cs[j];
    if (sj.start == NONE) continue;
    if (sj.status != ST_OK) bad = 1;
    if (j == c0) continue;
    int p = (int)j - 1;
    for (uint32_t g = 0; g < fd.n_chunks && p >= (int)c0 && cs[p].start == NONE; g++) p--;
    if (p < (int)c0) {
      bad = 1;
      continue;
    }
    const ChunkState sp = cs[p];
    if (sp.status != ST_OK || (sp.flags & CS_FINAL) || sp.end != sj.start) bad = 1;
  }
  __syncthreads();
  if (bad && tid < 64) {
    // sequential walk by one wave: re-decode every chunk whose start is not
    // where the previous accepted chunk ended
    uint64_t cur = NONE;
    bool fin = false;
    uint32_t repairs = 0;
    int32_t st = ST_OK;
    for (uint32_t j = c0; j < c1; j++) {
      uint64_t sj = uni64(cs[j].start);
      if (sj == NONE) continue;
      if (fin) {
        if (tid == 0) {
          cs[j].start = NONE;
          cs[j].len = 0;
          cs[j].flags = CS_EMPTY;
          cs[j].status = ST_OK;
        }
        continue;
      }
      if (j != c0 && sj != cur) {
        repairs++;
        uint32_t nx;
        uint64_t stop = uni64(next_start(fd, cs, j, true, &nx));
        if (cur >= stop) {
          if (tid == 0) {
            cs[j].start = cur;
            cs[j].end = cur;
            cs[j].len = 0;
            cs[j].flags = CS_REPAIRED;
            cs[j].status = ST_OK;
          }
        } else {
          redecode_chunk<WIN>(sh, fd, chunks[j], cs, pool, j, cur, stop);
        }
      }
      const int32_t sj_status = uni(cs[j].status);
      if (sj_status != ST_OK) {
        st = sj_status;
        if (sj_status == ST_DATA) break;
      }
      cur = uni64(cs[j].end);
      fin = (uni(cs[j].flags) & CS_FINAL) != 0;
    }
    if (st == ST_OK && !fin) st = ST_DATA;  // stream ends without a final block
    if (tid == 0) {
      fs[f].status = st;
      fs[f].n_repairs = repairs;
    }
  }
  __syncthreads();
  // exclusive scan of lengths in chunk order; per-file statistics
  uint64_t carry = 0;
  uint64_t nsyms = 0, nph = 0, nblk = 0;
  uint32_t nonempty = 0, ext = 0, retries = 0, overflow = 0;
  uint64_t last_end = NONE;
  uint32_t last_flags = 0;
  for (uint32_t base = c0; base < c1; base += blockDim.x) {
    const uint32_t j = base + tid;
    uint64_t L = 0;
    if (j < c1) {
      const ChunkState sj = cs[j];
      if (sj.start != NONE) {
        L = sj.len;
        nonempty++;
        nsyms += sj.n_syms;
        nph += sj.n_placeholders;
        nblk += sj.n_blocks;
        if (sj.flags & CS_EXTENDED) ext++;
        if (sj.flags & CS_OVERFLOW) overflow++;
      }
      retries += sj.retries;
    }
    part[tid] = L;
    __syncthreads();
    // Hillis-Steele inclusive scan (256 entries)
    for (int o = 1; o < 256; o <<= 1) {
      uint64_t a = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      __syncthreads();
    }
    if (j < c1) {
      const uint64_t off = carry + part[tid] - L;
      cs[j].out_off = off;
      cs[j].valid = (uint32_t)(off < WINDOW ? off : WINDOW);
    }
    carry += part[255];
    __syncthreads();
  }
  // reductions of the statistics
  part[tid] = nsyms;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_syms = part[0];
  __syncthreads();
  part[tid] = nph;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_ph = part[0];
  __syncthreads();
  part[tid] = nblk | ((uint64_t)nonempty << 40);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_blk = part[0] & ((1ull << 40) - 1), tot_ne = part[0] >> 40;
  __syncthreads();
  part[tid] = (uint64_t)ext | ((uint64_t)retries << 20) | ((uint64_t)overflow << 42);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t packed = part[0];
  if (tid == 0) {
    // the last accepted chunk must end on the final block, right before the trailer
    for (int j = (int)c1 - 1; j >= (int)c0; j--)
      if (cs[j].start != NONE) {
        last_end = cs[j].end;
        last_flags = cs[j].flags;
        break;
      }
    int32_t st = fs[f].status;
    const uint32_t ovf = (uint32_t)(packed >> 42);
    if (st == ST_OK) {
      if (!(last_flags & CS_FINAL)) st = ST_DATA;
      else if (((last_end + 7) >> 3) + 8 != fd.comp_len) st = ST_UNSUPPORTED;
      else if (ovf) st = ST_CAPACITY;
      else if (carry > fd.out_cap) st = ST_CAPACITY;
      else if ((uint32_t)carry != fd.isize) st = ST_SIZE;
    }
    fs[f].status = st;
    fs[f].out_len = carry;
    fs[f].out_needed = carry;
    fs[f].n_syms = tot_syms;
    fs[f].n_placeholders = tot_ph;
    fs[f].n_blocks = tot_blk;
    fs[f].n_nonempty = (uint32_t)tot_ne;
    fs[f].n_extended = (uint32_t)(packed & 0xFFFFF);
    fs[f].n_retries = (uint32_t)((packed >> 20) & 0x3FFFFF);
    fs[f].overflow = ovf;
  }
}

// ---------------------------------------------------------------------------
// k_propagate: one workgroup per file walks the accepted chunks in order.
// w_next[k] = t < 256 ? t : w[t & 0x7FFF], t = symbol k of the last 32768
// of (w_hat_i ++ D_i); the first chunk's window is unknown (zero).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_propagate(const FileDesc *files, const ChunkDesc *chunks,
                                                    const ChunkState *cs, const FileState *fs, uint8_t *wins,
                                                    const uint16_t *pool) {
  __shared__ uint8_t wbuf[2][WINDOW];
  const uint32_t f = blockIdx.x;
  const FileDesc fd = files[f];
  if (fs[f].status != ST_OK) return;
  const int tid = (int)threadIdx.x;
  const uint32_t c0 = fd.first_chunk, c1 = fd.first_chunk + fd.n_chunks;
  for (int k = tid; k < (int)WINDOW; k += blockDim.x) wbuf[0][k] = 0;
  __syncthreads();
  int cur = 0;
  uint32_t j = c0;
  for (uint32_t g = 0; g < fd.n_chunks && j < c1 && cs[j].start == NONE; g++) j++;
  for (uint32_t step = 0; step < fd.n_chunks && j < c1; step++) {
    uint32_t jn = j + 1;
    for (uint32_t g = 0; g < fd.n_chunks && jn < c1 && cs[jn].start == NONE; g++) jn++;
    if (jn >= c1) break;
    const uint64_t L = cs[j].len;
    const uint16_t *Dj = pool + chunks[j].sym_off;
    uint8_t *wo = wins + (uint64_t)jn * WINDOW;
    for (int k = tid; k < (int)WINDOW; k += blockDim.x) {
      const uint64_t q = L + (uint64_t)k;
      const uint32_t t = q < WINDOW ? (0x8000u | (uint32_t)q) : (uint32_t)Dj[q - WINDOW];
      const uint8_t b = t < 256u ? (uint8_t)t : wbuf[cur][t & 0x7FFFu];
      wbuf[cur ^ 1][k] = b;
      wo[k] = b;
    }
    __syncthreads();
    cur ^= 1;
    j = jn;
  }
}

// ---------------------------------------------------------------------------
// k_tilescan: one workgroup; tiles[j] = translate tiles before chunk j over
// the whole batch (files whose status is not OK contribute none).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tilescan(const ChunkDesc *chunks, const ChunkState *cs, const FileState *fs,
                                                   uint32_t n, uint64_t *tiles) {
  __shared__ uint64_t part[1024];
  const int tid = (int)threadIdx.x;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < n; base += 1024) {
    const uint32_t j = base + (uint32_t)tid;
    uint64_t T = 0;
    if (j < n && cs[j].start != NONE && fs[chunks[j].file].status == ST_OK)
      T = (cs[j].len + TRANSLATE_TILE - 1) / TRANSLATE_TILE;
    part[tid] = T;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      uint64_t a = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      __syncthreads();
    }
    if (j < n) tiles[j] = carry + part[tid] - T;
    carry += part[1023];
    __syncthreads();
  }
  if (tid == 0) tiles[n] = carry;
}

// ---------------------------------------------------------------------------
// k_translate: out[o_i + p] = D_i[p] < 256 ? D_i[p] : w_i[D_i[p] & 0x7FFF].
// Tiles of TRANSLATE_TILE symbols; a persistent grid walks them.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_translate(const FileDesc *files, const ChunkDesc *chunks, const ChunkState *cs,
                                                   FileState *fs, const uint64_t *tiles, uint32_t n,
                                                   const uint8_t *wins, const uint16_t *pool, Counters *ctr) {
  __shared__ uint32_t s_item;
  const uint64_t total = tiles[n];
  for (uint64_t it = 0; it <= total; it++) {
    if (threadIdx.x == 0) s_item = atomicAdd(&ctr->translate_next, 1u);
    __syncthreads();
    const uint64_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    // chunk: the last j with tiles[j] <= item (chunks without tiles repeat the next value)
    uint32_t lo = 0, hi = n;
    for (int it = 0; it < 40 && hi - lo > 1; it++) {
      uint32_t mid = (lo + hi) >> 1;
      if (tiles[mid] <= item) lo = mid;
      else hi = mid;
    }
    const uint32_t j = lo;
    const ChunkState sj = cs[j];
    const FileDesc fd = files[chunks[j].file];
    const uint64_t p0 = (item - tiles[j]) * TRANSLATE_TILE;
    const uint64_t L = sj.len;
    const uint16_t *Dj = pool + chunks[j].sym_off;
    const uint8_t *wj = wins + (uint64_t)j * WINDOW;
    const uint32_t lim = 32768u - sj.valid;  // placeholders below this lie before the data start
    uint8_t *out = fd.out + sj.out_off;
    int err = 0;
    for (uint64_t g = p0 + 8ull * threadIdx.x; g < p0 + TRANSLATE_TILE && g < L; g += 8ull * blockDim.x) {
      const uint4 v = *reinterpret_cast<const uint4 *>(Dj + g);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int h = 0; h < 8; h++) {
        const uint64_t p = g + h;
        if (p < L) {
          const uint32_t t = (w[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
          uint32_t b;
          if (t < 256u) {
            b = t;
          } else {
            const uint32_t m = t & 0x7FFFu;
            if (t < 0x8000u || m < lim) err = 1;
            b = wj[m];
          }
          out[p] = (uint8_t)b;
        }
      }
    }
    if (err) atomicCAS(&fs[chunks[j].file].status, ST_OK, ST_DATA);
  }
}

// ---------------------------------------------------------------------------
// Host-callable launchers
// ---------------------------------------------------------------------------

}  // namespace gzgpu

using namespace gzgpu;

extern "C" {

hipError_t gzk_init(ChunkState *cs, uint32_t n_chunks, FileState *fs, uint32_t n_files, Counters *ctr,
                    hipStream_t st) {
  uint32_t n = n_chunks > n_files ? n_chunks : n_files;
  if (n < 16) n = 16;
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, cs, n_chunks, fs, n_files, ctr);
  return hipGetLastError();
}

hipError_t gzk_capacity(uint32_t n_files, const FileDesc *files, ChunkDesc *chunks, const ChunkState *cs,
                        uint32_t factor, hipStream_t st) {
  hipLaunchKernelGGL(k_capacity, dim3(n_files), dim3(256), 0, st, files, chunks, cs, factor);
  return hipGetLastError();
}

hipError_t gzk_scan(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs, const uint32_t *scan_list,
                    uint32_t n_scan, uint32_t groups, hipStream_t st) {
  if (n_scan == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(n_scan * groups), dim3(256), 0, st, files, chunks, cs, scan_list, n_scan, groups);
  return hipGetLastError();
}

#define GZ_WIN_SWITCH(win, CALL) \
  {                              \
    (void)(win);                 \
    constexpr int W = 32768;     \
    CALL;                        \
  }

hipError_t gzk_inflate(int win, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                       const uint32_t *order, uint32_t n, Counters *ctr, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_inflate<W>, dim3(grid), dim3(64), 0, st, files, chunks, cs, order, n, ctr,
                                        pool));
  return hipGetLastError();
}

hipError_t gzk_stitch(int win, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                      uint32_t n, Counters *ctr, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_stitch<W>, dim3(grid), dim3(64), 0, st, files, chunks, cs, n, ctr, pool));
  return hipGetLastError();
}

hipError_t gzk_finalize(int win, uint32_t n_files, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                        FileState *fs, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_finalize<W>, dim3(n_files), dim3(256), 0, st, files, chunks, cs, fs, pool));
  return hipGetLastError();
}

hipError_t gzk_tilescan(const ChunkDesc *chunks, const ChunkState *cs, const FileState *fs, uint32_t n, uint64_t *tiles,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_tilescan, dim3(1), dim3(1024), 0, st, chunks, cs, fs, n, tiles);
  return hipGetLastError();
}

hipError_t gzk_propagate(uint32_t n_files, const FileDesc *files, const ChunkDesc *chunks, const ChunkState *cs,
                         const FileState *fs, uint8_t *wins, const uint16_t *pool, hipStream_t st) {
  hipLaunchKernelGGL(k_propagate, dim3(n_files), dim3(1024), 0, st, files, chunks, cs, fs, wins, pool);
  return hipGetLastError();
}

hipError_t gzk_translate(uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, const ChunkState *cs,
                         FileState *fs, const uint64_t *tiles, uint32_t n, const uint8_t *wins, const uint16_t *pool,
                         Counters *ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_translate, dim3(grid), dim3(256), 0, st, files, chunks, cs, fs, tiles, n, wins, pool, ctr);
  return hipGetLastError();
}

}  // extern "C"
