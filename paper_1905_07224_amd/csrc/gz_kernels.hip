// HIP kernels of the two-pass gzip path (gfx950).
//
//   k_init       clear per-chunk and per-file state (a kernel, so the whole
//                sequence can be captured in a graph)
//   k_scan       block-start search (Section VI-A, Appendix A): stage 1 on
//                every candidate bit (32 per lane per step), stage 2 (the
//                code tables) on the survivors, one survivor per lane
//   k_capacity   each chunk's symbol region from the span to the next start
//   k_inflate    pass 1, decompress(C_i, w_hat_i) (Section VI-C): one wave per
//                chunk from a persistent work queue, tables and the recent
//                history in LDS, 16-bit symbols to HBM; the trial block and
//                the confirmation blocks of the start checks
//   k_confirm    confirmation blocks owed past a chunk's stop (deferred)
//   k_redo       chunks whose deferred confirmation failed search again
//   k_stitch     chunks whose stop was not the next accepted start continue
//   k_finalize   stitch check, sequential repair when a start is off the
//                block chain, output offsets (exclusive scan of |D_i|)
//   k_tilescan   translate tiles and the list of chunks with a start
//   k_prop_*     pass 2a: windows resolved by a scan of composed maps over
//                segments of 64 chunks
//   k_translate  pass 2b: every U_j replaced by w_i[j], written to the output
//   k_crc        CRC-32 of every output (RFC 1952), checked by k_crc_final
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

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
static_assert(sizeof(InflateLDS<512>) <= inflate_lds_bytes(512) && sizeof(InflateLDS<1024>) <= inflate_lds_bytes(1024) &&
                  sizeof(InflateLDS<2048>) <= inflate_lds_bytes(2048) && sizeof(InflateLDS<4096>) <= inflate_lds_bytes(4096) && sizeof(InflateLDS<8192>) <= inflate_lds_bytes(8192) &&
                  sizeof(InflateLDS<16384>) <= inflate_lds_bytes(16384) &&
                  sizeof(InflateLDS<32768>) <= inflate_lds_bytes(32768),
              "decoder LDS larger than the occupancy estimate");

struct DecodeResult {
  int status;        // D_OK or failure
  bool confirmed;    // the check blocks all passed (or none were asked)
  bool final_seen;
  bool cut;          // the symbols outgrew the capacity: only those before cut_bit were stored
  uint64_t end;      // stop bit
  uint64_t len;      // symbols up to the stop
  uint32_t blocks;
  uint32_t pending;  // check blocks left for after the stop (deferred confirmation)
  // with cut: the last block boundary whose symbols all fit, and the symbols,
  // blocks, codes and (per lane) placeholders before it
  uint64_t cut_bit, cut_len, cut_syms;
  uint32_t cut_blocks, cut_nph;
};

// STORED: the trial block may be a stored block (chunks searched with
// FD_STORED_STARTS); false compiles the trial for dynamic blocks only.
template <int WIN, bool STORED = false>
struct Inflater {
  // The ring holds the last WIN symbols (WIN a power of two, 512..32768).
  // Symbols move to HBM in units of UNIT <= WIN / 2; fewer than UNIT are
  // unstored when a batch is issued and fewer than UNIT + 64 after it is
  // written, so no unstored symbol is overwritten.  A batch reads all its
  // sources before it writes any of its symbols, so a source pos - d + k with
  // d <= WIN is in the ring; an older one (only when WIN < 32768) lies below
  // pos - WIN <= stored - (WIN - UNIT), in a unit before the last one stored:
  // every unit store waits for the stores before it, so those are complete,
  // and the read bypasses the L1, which may still hold lines of an earlier
  // attempt at this chunk.
  static_assert(WIN >= 512 && WIN <= 32768 && (WIN & (WIN - 1)) == 0, "ring size");
  static constexpr uint32_t RMASK = WIN - 1;
  static constexpr uint32_t UNIT = WIN < 2 * FLUSH_UNIT ? WIN / 2 : FLUSH_UNIT;
  static constexpr uint32_t PER_LANE = UNIT / 64;  // symbols each lane moves: 8 (one uint4) or 4 (one uint2)
  using UnitVec = typename std::conditional<PER_LANE == 8, uint4, uint2>::type;
  static_assert(UNIT % 64 == 0 && (PER_LANE == 8 || PER_LANE == 4) && FLUSH_UNIT % UNIT == 0, "flush unit");

  InflateLDS<WIN> &sh;
  WaveBits br;
  uint16_t *D;       // chunk symbols in HBM
  uint64_t cap;      // symbol capacity
  uint64_t pos;      // symbols produced
  uint64_t flushed;  // symbols stored to HBM (multiple of UNIT)
  uint64_t nsyms;
  uint32_t nph;      // per lane placeholder count
  uint32_t nph_stop; // per lane placeholder count at the stop (symbols of D_i only)
  bool first;        // empty context
  bool ascii;        // checked blocks reject literals outside the ASCII set (text input)
  bool stored_ok;    // a stored block may be the trial block (FD_STORED_STARTS)
  bool over;         // capacity exceeded somewhere
  bool emit;         // false: blocks past the stop are only parsed and counted

  __device__ Inflater(InflateLDS<WIN> &s) : sh(s) {}
  __device__ __forceinline__ uint32_t sh_lit(uint32_t i) const { return sh.t.lit[i]; }
  __device__ __forceinline__ uint32_t sh_dist(uint32_t i) const { return sh.t.dist[i]; }

  __device__ __forceinline__ void flush_unit() {
    // earlier unit stores complete (vmcnt 0) before this one is issued
    if (WIN < 32768) __builtin_amdgcn_s_waitcnt(0xF70);
    wave_sync();
    const int lane = lane_id();
    const uint64_t u = flushed;
    const UnitVec v = *reinterpret_cast<const UnitVec *>(&sh.ring[(u + PER_LANE * lane) & RMASK]);
    if (u + UNIT <= cap) {
      *reinterpret_cast<UnitVec *>(D + u + PER_LANE * lane) = v;
    } else {
      over = true;
    }
    flushed = u + UNIT;
  }
  __device__ __forceinline__ void maybe_flush() {
    while (pos > flushed && pos - flushed >= UNIT) flush_unit();
  }
  __device__ void flush_all() {
    while (flushed < pos) flush_unit();
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
        bad = check && ascii && !ascii_text(c);
        if (emit) sh.ring[(pos + (uint32_t)lane) & RMASK] = (uint16_t)c;
      }
      if (__ballot(bad)) return D_ASCII;
      pos += min(64u, n - k0);
      if (emit) maybe_flush();
    }
    br.pos += 8ull * n;
    return D_OK;
  }

  // Output of one batch: lane l < j describes symbol pos + l.  A value
  // >= REF_LIT is a literal (low 16 bits); otherwise it is l - distance, a
  // lane of this batch when >= 0, else a symbol produced before the batch.
  static constexpr int32_t REF_LIT = 0x10000;

  // A batch is resolved in two steps so that its HBM reads overlap the
  // decoding of the next one.  issue(): sources before the batch come from
  // the ring, from HBM (loads left in flight), or are the placeholders U_j
  // before a chunk (a distance past the start of the first chunk is invalid
  // data); sources in the batch are earlier lanes.  finish(): pointer
  // jumping over those (a lane whose source is still open takes that lane's
  // source, so after k rounds every chain of up to 2^k links is closed), then
  // the symbols go to the ring.  finish() of one batch always precedes
  // issue() of the next, so every ring read sees all earlier symbols.
  uint32_t pj;   // symbols of the pending batch (0: none)
  uint32_t pval; // per lane: its symbol, or (pp != lane) not yet known
  uint32_t plv;  // per lane: the HBM load in flight (used where pfar has the lane's bit)
  uint64_t pfar;
  int32_t pp;    // per lane: lane whose symbol this one copies, itself when known

  __device__ __forceinline__ int issue(int32_t ref, uint32_t j) {
    const int lane = lane_id();
    wave_sync();
    // every lane works out every case and selects one, with no divergent
    // branch (whose exec-mask bookkeeping would cost more than the cases)
    const bool act = lane < (int)j;
    const bool lit = ref >= REF_LIT;
    const bool back = act && !lit && ref < 0;  // a symbol produced before the batch
    const int64_t a = (int64_t)pos + ref;
    const bool before = back && a < 0;         // a placeholder U_j before the chunk
    const bool near = WIN == 32768 || ref >= -(int32_t)WIN;  // a >= pos - WIN: in the ring
    bool far = back && !before && !near;
    // the ring slot of a (the index is masked, so lanes that do not need it
    // read some slot of the ring, unused)
    const uint32_t rv = (uint32_t)sh.ring[((uint32_t)pos + (uint32_t)ref) & RMASK];
    const uint32_t val = lit ? ((uint32_t)ref & 0xFFFFu) : before ? (0x8000u | (uint32_t)(a + WINDOW)) : rv;
    const int32_t p = act && !lit && ref >= 0 ? ref : lane;
    if (first && __ballot(before)) return D_FAR;
    // every lane loads (element 0 where no HBM source is needed), so the load
    // writes its register directly and is waited for only in finish()
    // (past capacity nothing was stored: that chunk fails with a capacity
    // status, so any value will do)
    if (far && (uint64_t)a >= cap) far = false;
    uint32_t lv = 0;
    const uint64_t fm = WIN < 32768 ? __ballot(far) : 0ull;
    // the aligned dword that holds the symbol (D is 4-byte aligned)
    if (fm)
      lv = __hip_atomic_load(reinterpret_cast<const uint32_t *>(D) + (far ? (a >> 1) : 0), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    pval = far ? (uint32_t)(a & 1) << 4 : val;  // far lanes: which half
    plv = lv;
    pfar = fm;
    pp = p;
    pj = j;
    return D_OK;
  }

  __device__ __forceinline__ int finish() {
    if (pj == 0) return D_OK;
    const int lane = lane_id();
    uint32_t val = (pfar >> lane) & 1ull ? (plv >> pval) & 0xFFFFu : pval;
    int32_t p = pp;
    for (int it = 0; it < 8; it++) {
      if (__ballot(p != lane) == 0) break;
      const uint32_t vs = __shfl(val, p);
      const int32_t ps = __shfl(p, p);
      if (p != lane) {
        if (ps == p) {
          val = vs;
          p = lane;
        } else {
          p = ps;
        }
      }
    }
    if (__ballot(p != lane)) return D_BAD;  // unreachable: chains are shorter than 64
    if (lane < (int)pj) {
      sh.ring[(pos + (uint32_t)lane) & RMASK] = (uint16_t)val;
      nph += val >> 15;
    }
    pos += pj;
    pj = 0;
    maybe_flush();
    return D_OK;
  }

  // Output of one batch, pipelined (parse-only past the stop: counted only).
  __device__ __forceinline__ int put_batch(int32_t ref, uint32_t j) {
    if (!emit) {
      pos += j;
      return D_OK;
    }
    const int r = finish();
    if (r != D_OK) return r;
    return issue(ref, j);
  }

  // A symbol whose code is longer than the lookup tables, decoded alone at
  // br.pos: *len_out = 0 for a literal (stored in *lit), 0xFFFFFFFF for
  // end-of-block, else a match of *len_out symbols at *dist_out.
  __device__ int slow_symbol(bool check, uint32_t *lit, uint32_t *len_out, uint32_t *dist_out) {
    const uint64_t v = br.next();
    uint32_t e = uni32(sh.t.lit[v & ((1u << LIT_BITS) - 1u)]);
    if (e == TOK_SLOW) e = decode_long<LIT_BITS, TREE_LIT>(v, &sh.t.li, sh.t.lsorted);
    const uint32_t nout = (e >> 8) & 511u, cl = e & 15u;
    nsyms++;
    if (nout == 1u) {
      if (check && ascii && (e & TOK_NONASCII)) return D_ASCII;
      *lit = (e >> 17) & 255u;
      *len_out = 0;
      br.skip(cl);
      return br.past_end() ? D_TRUNC : D_OK;
    }
    if ((e & ~255u) == TOK_EOB) {
      *len_out = 0xFFFFFFFFu;
      br.skip(cl);
      return br.past_end() ? D_TRUNC : D_OK;
    }
    if (nout != 0u) return D_BAD;
    const uint32_t ex = (e >> 4) & 15u;
    const uint32_t len = (e >> 17) + ((uint32_t)(v >> cl) & ((1u << ex) - 1u));
    const uint32_t used = cl + ex;
    const uint64_t v2 = v >> used;
    uint32_t ed = uni32(sh.t.dist[v2 & ((1u << DIST_BITS) - 1u)]);
    if (((ed >> 4) & 15u) == K_LONG) ed = decode_long<DIST_BITS, TREE_DIST>(v2, &sh.t.di, sh.t.dsorted);
    if (((ed >> 4) & 15u) != K_LEN) return D_BAD;
    const uint32_t dl = ed & 15u, dex = (ed >> 8) & 255u;
    *dist_out = (ed >> 16) + ((uint32_t)(v2 >> dl) & ((1u << dex) - 1u));
    *len_out = len;
    br.skip(used + dl + dex);
    return br.past_end() ? D_TRUNC : D_OK;
  }

  // Token words of one lookup round (per lane k: the token that would start
  // at bit offset k): bits 7..0 the bits it uses (at most 48), bits 16..8
  // its output length (1: a literal), bits 31..17 the literal byte or the
  // match distance minus one (0..32767).  The walk adds whole token words to
  // its packed (output symbols << 8 | bit offset) counter: the low 17 bits
  // hold the counter (fewer than 64 + 258 symbols, offsets below 256), the
  // bits above only collect the payloads and are never read.  A special
  // token (TOK_*) has length 448: added to fewer than 64 symbols it sets
  // bits 14..16 of the counter, which ends any walk, and stays below bit 17.
  // Literal and special tokens are literal/length table entries as they
  // stand; only a length code's token is assembled here.
  __device__ __forceinline__ static bool tok_special(uint32_t t) { return (t & TOK_SPECIAL) == TOK_SPECIAL; }

  // The token word at bit offset k of a lookup round, from the 64 stream
  // bits at that offset (w: bits k .. k + 63) and its two table entries
  // (e: literal/length, ed: distance, looked up at the bits after the
  // length's extra bits).  Straight-line code: the match case is computed
  // for every lane and selected where e is a length code.
  template <bool CHECK>
  __device__ __forceinline__ static uint32_t token_word(uint64_t w, uint32_t e, uint32_t ed, bool ascii) {
    const uint32_t w0 = (uint32_t)w;
    const uint32_t cl = e & 15u, ex = (e >> 4) & 15u;
    const uint32_t u = cl + ex;
    const uint32_t dl = ed & 15u, dex = (ed >> 8) & 15u;
    const uint32_t len = (e >> 17) + ((w0 >> cl) & ((1u << ex) - 1u));
    const uint32_t dist = (ed >> 16) + ((uint32_t)(w >> (u + dl)) & ((1u << dex) - 1u));
    const uint32_t wm = ((ed >> 4) & 15u) == K_LEN ? (u + dl + dex) | (len << 8) | ((dist - 1u) << 17) : TOK_SLOW;
    uint32_t t = (e & (511u << 8)) == 0u ? wm : e;
    // only literal entries have bit 31 set
    if (CHECK) t = (ascii && (e & TOK_NONASCII)) ? TOK_ASCII : t;
    return t;
  }

  // Token words at bit offsets k (wa) and k + 64 (wb): both
  // literal/length lookups, then both distance lookups.
  template <bool CHECK>
  __device__ __forceinline__ void token_pair(uint64_t wa, uint64_t wb, uint32_t &ta, uint32_t &tb) const {
    const uint32_t LMASK = (1u << LIT_BITS) - 1u, DMASK = (1u << DIST_BITS) - 1u;
    const uint32_t ea = sh_lit((uint32_t)wa & LMASK);
    const uint32_t eb = sh_lit((uint32_t)wb & LMASK);
    // the bits after a length code's extra bits (elsewhere unused)
    const uint32_t ua = (ea & 15u) + ((ea >> 4) & 15u), ub = (eb & 15u) + ((eb >> 4) & 15u);
    const uint32_t eda = sh_dist((uint32_t)(wa >> ua) & DMASK);
    const uint32_t edb = sh_dist((uint32_t)(wb >> ub) & DMASK);
    ta = token_word<CHECK>(wa, ea, eda, ascii);
    tb = token_word<CHECK>(wb, eb, edb, ascii);
  }

  // Huffman-coded block body until end-of-block (section 3.2.5), decoded in
  // rounds of 128 bit offsets.  Lane k reads the 64 stream bits at offsets k
  // and k + 64 from br.pos and decodes the tokens that would start there:
  // literal/length code, extra length bits, distance code and extra distance
  // bits (at most 48 bits, RFC 1951 section 3.2.5), with one lookup in each
  // table.  The scalar walk then follows the real tokens from offset 0 (each
  // one bit count further) while they start below offset 128, recording only
  // where each starts in the batch of up to 64 output symbols; then every
  // lane finds its token (the last start at or before it) and takes its
  // source from the token's word.  CHECK: literals must be ASCII text
  // (block-start trial and confirmation).
  //
  // A batch is not tied to a round: when the walk reaches the end of a round
  // before the batch has 64 symbols, the next round is decoded and the walk
  // goes on filling the same batch, so that the per-batch work (source
  // selection, pointer jumping, ring and HBM stores) is paid once per 64
  // symbols and not once per round.
  template <bool CHECK>
  __device__ int huffman(uint64_t size_cap, uint64_t blk0) {
    const int lane = lane_id();
    uint32_t tok0 = 0, tok1 = 0;  // token words at offsets lane and lane + 64
    uint32_t off = 0;   // bit offset of the walk from br.pos, where the round was decoded
    bool need = true;   // a round to be decoded at br.pos + off
    uint32_t rem = 0, mdist = 0;  // part of a match still to be produced
    // the batch being assembled: start lanes' token words, symbols so far,
    // and whether it began with the rest of a match (open: being assembled)
    uint32_t word = 0, jr = 0, cont = 0;
    bool open = false;
    // an iteration consumes at least one bit or produces 64 symbols (<= 258
    // per code): the remaining bits bound the iterations (a 32-bit count:
    // even a 4 GiB output takes far fewer than 2^32 iterations)
    const uint64_t budget64 = 8ull * (br.s.end_bits - br.pos + 64);
    const uint32_t budget = budget64 < 0xFFFFFFFFull ? (uint32_t)budget64 : 0xFFFFFFFFu;
    for (uint32_t it = 0;; it++) {
      if (it >= budget) return D_BAD;
      if (need) {
        br.pos += off;
        // past the end of the input (the bit reader reads zeros there)
        if (br.past_end()) return D_TRUNC;
        // the 64 bits at offsets k and k + 64
        uint64_t wa, wb;
        br.lane_windows(wa, wb);
        token_pair<CHECK>(wa, wb, tok0, tok1);
        off = 0;
        need = false;
      }
      // start lanes of the batch's tokens, and each start lane's token word
      // (the rest of a match begun in the last batch is the token at lane 0)
      // (a token word is never 0, so the start lanes are where word != 0)
      if (!open) {
        word = 0;
        jr = 0;  // output symbols of the tokens walked so far
        cont = min(rem, 1u);  // (an integer, not a lane mask)
        if (rem) {
          word = (uint32_t)GZ_WRITELANE((int)((2u << 8) | ((mdist - 1u) << 17)), 0, 0);
          jr = rem;
        }
        open = true;
      }
      // acc = jr << 8 | off; offsets below 64 come from tok0, the rest from
      // tok1 (a walk never returns below an offset it passed, so the two
      // halves are two loops).  Each step writes the token's word at lane jr
      // and adds the word; a special token adds 448 symbols, which ends the
      // walk, and is taken back out below.
      uint32_t acc = (jr << 8) | off;
      uint32_t t = 0;  // the last token walked
      if ((acc & 0x1C0C0u) == 0u) {
        do {
          t = (uint32_t)__builtin_amdgcn_readlane((int)tok0, (int)(acc & 63u));
          word = (uint32_t)GZ_WRITELANE((int)t, (int)((acc >> 8) & 63u), (int)word);
          acc += t;
        } while ((acc & 0x1C0C0u) == 0u);
      }
      if ((acc & 0x1C080u) == 0u) {
        do {
          t = (uint32_t)__builtin_amdgcn_readlane((int)tok1, (int)(acc & 63u));
          word = (uint32_t)GZ_WRITELANE((int)t, (int)((acc >> 8) & 63u), (int)word);
          acc += t;
        } while ((acc & 0x1C080u) == 0u);
      }
      uint32_t x = 0;  // the special token that stopped the walk, else 0
      if (tok_special(t)) {
        x = t;
        acc -= t;
        word = (uint32_t)GZ_WRITELANE(0, (int)((acc >> 8) & 63u), (int)word);
      }
      jr = (acc >> 8) & 511u;
      off = acc & 255u;
      if (x == 0u && jr < 64u && off >= 128u) {
        // the round is used up before the batch is full: the next round
        // continues the same batch
        need = true;
        continue;
      }
      open = false;
      const uint64_t starts = __ballot(word != 0u);
      // a token running past the batch continues in the next one (its
      // word is at the last start lane)
      const uint32_t j = jr < 64u ? jr : 64u;
      rem = jr - j;
      if (rem) mdist = ((uint32_t)__builtin_amdgcn_readlane((int)word, 63 - __builtin_clzll(starts)) >> 17) + 1u;
      nsyms += (uint32_t)__builtin_popcountll(starts) - cont;
      if (j) {
        // each lane's token: the last start at or before the lane
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const uint64_t m = starts & upto;
        const int src = 63 - (int)__builtin_clzll(m | 1ull);
        const uint32_t w = (uint32_t)__shfl((int)word, src);
        const int32_t ref = ((w >> 8) & 511u) == 1u ? (int32_t)(REF_LIT | ((w >> 17) & 255u))
                                                    : lane - (int32_t)((w >> 17) + 1u);
        const int r = put_batch(ref, j);
        if (r != D_OK) return r;
      }
      if (x) {
        if (x == TOK_ASCII) return D_ASCII;
        if ((x & ~255u) == TOK_EOB) {
          nsyms++;
          br.pos += off + (x & 255u);
          const int r = finish();
          if (r != D_OK) return r;
          return br.past_end() ? D_TRUNC : D_OK;
        }
        // TOK_SLOW or TOK_BADSYM: one symbol decoded alone (a bad one fails
        // there), then a new round
        br.pos += off;
        off = 0;
        need = true;
        uint32_t c = 0, len = 0, dist = 0;
        const int r = slow_symbol(CHECK, &c, &len, &dist);
        if (r != D_OK) return r;
        if (len == 0xFFFFFFFFu) return finish();
        if (len == 0) {
          const int r2 = put_batch(lane == 0 ? (int32_t)(REF_LIT | c) : 0, 1u);
          if (r2 != D_OK) return r2;
        } else {
          rem = len;
          mdist = dist;
        }
      } else if (off >= 128u) {
        need = true;
      }
      // only the trial block (a checked block) has a size bound
      if (CHECK && pos - blk0 >= size_cap) return D_SIZE;
    }
  }

  // One block.  check: ASCII literals (block-start confirmation); strict: the
  // candidate block itself (must be a non-final dynamic block with a complete
  // literal/length code and a size in (1 KiB, 4 MiB)).
  __device__ __forceinline__ int block(bool check, bool strict, bool *final_out) {
    const uint64_t v = br.next();
    const uint32_t bfinal = (uint32_t)(v & 1u), btype = (uint32_t)((v >> 1) & 3u);
    br.skip(3);
    if (br.past_end()) return D_TRUNC;
    *final_out = bfinal != 0;
    if (strict && (bfinal || !(btype == 2u || (STORED && btype == 0u && stored_ok)))) return D_STATIC;
    const uint64_t blk0 = pos;
    int r;
    if (btype == 0u) {
      r = stored(check);
    } else if (btype <= 2u) {
      if (btype == 1u) {
        fixed_tables(sh.t);
        r = D_OK;
      } else {
        // with no distance codes the distance table holds only invalid
        // entries, so a length code fails as the format requires
        bool nd = false;
        r = read_dynamic_tables(br, sh.t, strict, true, &nd);
      }
      if (r == D_OK) {
        const uint64_t cap_sz = strict ? (4ull << 20) : ~0ull;
        r = check ? huffman<true>(cap_sz, blk0) : huffman<false>(cap_sz, blk0);
      }
    } else {
      r = D_BAD;
    }
    if (r == D_OK && strict && !(pos - blk0 > 1024u && pos - blk0 < (4ull << 20))) r = D_SIZE;
    return r;
  }

  // Decode whole blocks from bit `start`, with `pos` symbols already produced,
  // until the first block header at or past `stop` (or a final block).  The
  // first `check_blocks` blocks are the block-start trial and confirmation; if
  // the stop comes first they are still decoded (parsed and checked, not
  // stored), then the stop is reported -- unless `defer`: then decoding ends
  // at the stop and the check blocks still owed are returned in `pending`
  // (the blocks after the stop are the next chunks' first blocks, which
  // those chunks decode with the same checks).
  //
  // cut_ok: when the symbols outgrow the capacity, the decode goes on to its
  // stop parsing only (so the checks and the stop are as without the cut),
  // and the last block boundary whose symbols all fit is reported (res.cut,
  // cut_*): every symbol before it is stored, and the caller continues from
  // there once the room is known.
  __device__ __forceinline__ DecodeResult run(uint64_t start, uint64_t stop, uint32_t check_blocks, bool defer = false,
                                              bool cut_ok = false) {
    DecodeResult res;
    res.status = D_OK;
    res.confirmed = check_blocks == 0;
    res.final_seen = false;
    res.cut = false;
    res.end = NONE;
    res.len = 0;
    res.blocks = 0;
    res.pending = 0;
    br.init(start);
    uint32_t nb = 0;
    // the last block boundary whose symbols fit the capacity (every symbol
    // below the capacity is stored once the decode has gone past it)
    res.cut_bit = start;
    res.cut_len = pos;
    res.cut_syms = nsyms;
    res.cut_blocks = 0;
    res.cut_nph = nph;
    // a block header is at least 3 bits: the remaining bits bound the blocks
    const uint64_t budget = (br.s.end_bits - br.pos) / 3 + 2;
    for (uint64_t it = 0;; it++) {
      if (it > budget) {
        res.status = D_BAD;
        break;
      }
      if (!res.cut && res.end == NONE) {
        if (pos <= cap) {
          res.cut_bit = br.pos;
          res.cut_len = pos;
          res.cut_syms = nsyms;
          res.cut_blocks = nb;
          res.cut_nph = nph;
        } else if (cut_ok) {
          res.cut = true;
          emit = false;  // parse only from here: nothing past the boundary is stored
        }
      }
      if (res.end == NONE && br.pos >= stop) {
        res.end = br.pos;
        res.len = pos;
        nph_stop = nph;
        if (defer) {
          res.pending = nb < check_blocks ? check_blocks - nb : 0u;
          break;
        }
        // the confirmation blocks still to come are not part of this chunk:
        // their symbols are checked and counted but not stored
        flush_all();
        emit = false;
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
    if (emit) flush_all();
    return res;
  }

  // Confirmation blocks decoded on their own: `need` blocks from bit `start`
  // with the checks of the confirmation (ASCII literals; the trial block's
  // stricter rules do not apply), parsed only; a final block ends them.
  __device__ int confirm(uint64_t start, uint32_t need) {
    emit = false;
    first = false;
    br.init(start);
    for (uint32_t nb = 0; nb < need; nb++) {
      bool fin = false;
      const int r = block(true, false, &fin);
      if (r != D_OK) return r;
      if (fin) break;
    }
    return D_OK;
  }
};

template <int WIN, bool STORED>
__device__ __forceinline__ void inflater_setup(Inflater<WIN, STORED> &inf, const FileDesc &fd, const ChunkDesc &cd,
                                               uint16_t *pool) {
  inf.br.s.init(fd.comp, fd.comp_len);
  inf.D = pool + cd.sym_off;
  inf.cap = cd.sym_cap;
  inf.pos = 0;
  inf.flushed = 0;
  inf.nsyms = 0;
  inf.nph = 0;
  inf.nph_stop = 0;
  inf.first = (cd.flags & (CF_FIRST | CF_CARRIED)) == CF_FIRST;
  inf.ascii = (fd.mode & FD_BINARY) == 0u;
  inf.stored_ok = (fd.mode & FD_STORED_STARTS) != 0u;
  inf.over = false;
  inf.emit = true;
  inf.pj = 0;
}

// Next chunk of the same file that has a start (scan candidate or accepted);
// after the last one, the segment's stop (NONE for a whole member).
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
  return fd.stop_bit;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Decode chunk c from scratch (pass 1 for one chunk).
// defer: confirmation blocks past the stop are left to k_confirm.  from:
// NONE to start at the scan candidate, else the first bit to search a
// candidate from (a candidate rejected by k_confirm is redone from the next).
// STORED: stored blocks may be starts (FD_STORED_STARTS); false compiles the
// search and the trial block for dynamic starts only.
template <int WIN, bool STORED>
__device__ __forceinline__ void inflate_chunk(InflateLDS<WIN> &sh, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                              uint16_t *pool, uint32_t c, bool defer, uint64_t from) {
  const int lane = lane_id();
  const ChunkDesc cd = chunks[c];
  const FileDesc fd = files[cd.file];
  const bool first = (cd.flags & CF_FIRST) != 0;
  uint64_t b = first ? fd.payload_bit : uni64(cs[c].cand);
  const uint64_t stop = first || b != NONE ? uni64(next_start(fd, cs, c, false, nullptr)) : NONE;
  Inflater<WIN, STORED> inf(sh);
  // search the next candidate from `search` at the top of an attempt (one
  // call site of the search, for code size)
  uint64_t search = !first && from != NONE ? from : NONE;
  uint32_t retries = 0;
  uint32_t n1 = 0, n2 = 0, trial_rej = 0, conf_rej = 0;  // search statistics of this call
  // each retry moves the candidate forward by at least one bit
  const uint64_t max_tries = cd.hi_bit - cd.lo_bit + 2;
  for (uint64_t tries = 0;; tries++) {
    if (search != NONE) {
      Src src;
      src.init(fd.comp, fd.comp_len);
      b = wave_find_start<STORED>(src, search, cd.hi_bit, sh.t, &n1, &n2, fd.mode);
      search = NONE;
    }
    if (tries > max_tries) b = NONE;
    if (b == NONE || (!first && b >= cd.hi_bit)) {
      if (lane == 0) {
        cs[c].start = NONE;
        cs[c].found = NONE;
        cs[c].end = NONE;
        cs[c].len = 0;
        cs[c].flags = CS_EMPTY;
        cs[c].retries = retries;
        cs[c].status = ST_OK;
        cs[c].pad = 0;
        cs[c].stage1 += n1;
        cs[c].stage2 += n2;
        cs[c].trial_rej += trial_rej;
        cs[c].confirm_rej += conf_rej;
      }
      return;
    }
    inflater_setup(inf, fd, cd, pool);
    // a probe stops after the first block (and its confirmation); other
    // chunks that outgrow their capacity stop at a block boundary and are
    // continued by the stitch pass, with the room of the empty chunks after
    // them (a rejected candidate leaves its chunk empty)
    const bool probe = (fd.mode & FD_PROBE) != 0;
    DecodeResult r = inf.run(b, probe ? b + 1 : stop, first ? 0u : 6u, defer, !probe);
    if (r.status != D_OK && (first || r.blocks >= 6u)) {
      if (lane == 0) {
        cs[c].start = b;
        cs[c].found = b;
        cs[c].end = r.end;
        cs[c].len = r.len;
        cs[c].status = ST_DATA;
        cs[c].flags = 0;
        cs[c].retries = retries;
        cs[c].pad = 0;
        cs[c].stage1 += n1;
        cs[c].stage2 += n2;
        cs[c].trial_rej += trial_rej;
        cs[c].confirm_rej += conf_rej;
      }
      return;
    }
    if (r.status == D_OK) {
      // a cut decode keeps what was stored: the stitch pass continues it
      uint32_t ph = wave_sum(r.cut ? r.cut_nph : inf.nph_stop);
      bool overflow = !r.cut && inf.over && r.len > cd.sym_cap;
      if (lane == 0) {
        cs[c].start = b;
        cs[c].found = b;
        cs[c].end = r.end;
        cs[c].len = r.cut ? r.cut_len : r.len;
        cs[c].cut_bit = r.cut ? r.cut_bit : NONE;
        cs[c].status = overflow ? ST_CAPACITY : ST_OK;
        cs[c].needed = overflow ? r.len : 0;
        cs[c].flags = (r.final_seen ? CS_FINAL : 0u) | (overflow ? CS_OVERFLOW : 0u) | (r.cut ? CS_CUT : 0u);
        // blocks decoded to the stop (the deferred confirmation counts them)
        cs[c].n_blocks = r.blocks;
        cs[c].cut_blocks = r.cut ? r.cut_blocks : 0u;
        cs[c].n_syms = r.cut ? r.cut_syms : inf.nsyms;
        cs[c].n_placeholders = ph;
        cs[c].retries = retries;
        cs[c].pad = r.pending;
        cs[c].stage1 += n1;
        cs[c].stage2 += n2;
        cs[c].trial_rej += trial_rej;
        cs[c].confirm_rej += conf_rej;
      }
      return;
    }
    // the candidate failed the trial decode or the confirmation: next one
    retries++;
    if (r.blocks == 0) trial_rej++;
    else conf_rej++;
    search = b + 1;
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
    z.found = NONE;
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
    z.stage1 = 0;
    z.stage2 = 0;
    z.trial_rej = 0;
    z.confirm_rej = 0;
    z.cut_bit = NONE;
    z.cut_blocks = 0;
    z.pad2 = 0;
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
// [lo_bit, hi_bit) passing the static checks.  A wave covers 2048 candidate
// bits per step, one aligned dword per lane.  The header fields are tested
// for all 32 bits of a dword at once; the positions that pass them (about
// one in nine, at most eleven per dword) are compacted into a list in bit
// order and their code-length codes tested 64 at a time, one per lane, so
// that no lane idles while another works through its dword.  The
// survivors, rare, are queued in bit order; every
// SCAN_BATCH of them (and the rest at the end) are checked at once, one per
// lane (the full table check), and the first that passes is the wave's
// answer.  `groups` workgroups share one chunk and its 4 waves each take
// steps in an interleaved order; a step is skipped once a passing candidate
// before it is known.
// ---------------------------------------------------------------------------

constexpr uint32_t SCAN_BATCH = 64;

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void k_scan(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                              const uint32_t *scan_list, uint32_t n_scan, uint32_t groups) {
  __shared__ uint8_t k3[512];
  __shared__ uint8_t cltab[4][128 * 64] __attribute__((aligned(16)));  // per lane code-length tables, per wave
  __shared__ unsigned long long queue[4][2 * SCAN_BATCH];  // per wave: survivors in bit order
  kraft3_fill(k3, (int)threadIdx.x, (int)blockDim.x);
  __syncthreads();
  const uint32_t item = blockIdx.x / groups, g = blockIdx.x % groups;
  if (item >= n_scan) return;
  const uint32_t c = scan_list[item];
  const ChunkDesc cd = chunks[c];
  Src s;
  s.init(files[cd.file].comp, files[cd.file].comp_len);
  const uint32_t mode = uni(files[cd.file].mode);
  const uint32_t wave = uni32(threadIdx.x >> 6);
  const int lane = lane_id();
  unsigned long long *cand = (unsigned long long *)&cs[c].cand;
  unsigned long long *q = queue[wave];
  uint32_t nq = 0;  // queued survivors
  // check the first k queued survivors, one per lane: true when one passed
  // (its bit went to the chunk's candidate); else they are dropped
  auto check = [&](uint32_t k) -> bool {
    wave_sync();
    const uint64_t cur = uni64(__hip_atomic_load(cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t b = (uint32_t)lane < k ? (uint64_t)q[lane] : NONE;
    const bool tried = b < cur;
    const bool ok = tried && lane_tables_ok(s, b, cltab[wave], lane, mode);
    const uint64_t m = __ballot(ok);
    const uint32_t n_tried = (uint32_t)__builtin_popcountll(__ballot(tried));
    if (lane == 0 && n_tried) {
      atomicAdd(&cs[c].stage1, n_tried);
      atomicAdd(&cs[c].stage2, (uint32_t)__builtin_popcountll(m));
    }
    if (m) {
      const uint64_t bb = readlane64(b, __ffsll((unsigned long long)m) - 1);
      if (lane == 0) atomicMin(cand, (unsigned long long)bb);
      return true;
    }
    const uint64_t rest = (uint32_t)lane + k < nq ? (uint64_t)q[lane + k] : 0ull;
    wave_sync();
    if ((uint32_t)lane + k < nq) q[lane] = rest;
    nq -= k;
    return false;
  };
  // aligned-view dwords holding the range
  const int64_t mb = 8 * (int64_t)s.mis;
  const int64_t W0 = ((int64_t)cd.lo_bit + mb) >> 5;
  const int64_t W1 = ((int64_t)cd.hi_bit + mb + 31) >> 5;
  const uint64_t steps = (uint64_t)(W1 - W0 + 63) / 64;
  bool found = false;
  for (uint64_t t = (uint64_t)g + (uint64_t)groups * wave; t < steps && !found; t += (uint64_t)groups * 4u) {
    const int64_t Wt = W0 + 64 * (int64_t)t;
    const uint64_t first_bit = (uint64_t)std::max<int64_t>(32 * Wt - mb, (int64_t)cd.lo_bit);
    // the step's 67 dwords: one per lane and the three after them (lanes 0..2),
    // loaded together with the chunk's candidate so far; lane l takes dwords
    // W + 1 .. W + 3 from the lanes after it
    const int64_t W = Wt + lane;
    const uint32_t x0 = s.dw(W);
    const uint32_t xt = lane < 3 ? s.dw(Wt + 64 + lane) : 0u;
    const uint64_t cur = uni64(__hip_atomic_load(cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (cur <= first_bit) break;
    const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)xt, 0);
    const uint32_t t1 = (uint32_t)__builtin_amdgcn_readlane((int)xt, 1);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_readlane((int)xt, 2);
    const uint32_t n1 = (uint32_t)__shfl((int)x0, (lane + 1) & 63);
    const uint32_t n2 = (uint32_t)__shfl((int)x0, (lane + 2) & 63);
    const uint32_t n3 = (uint32_t)__shfl((int)x0, (lane + 3) & 63);
    const uint32_t x1 = lane < 63 ? n1 : t0;
    const uint32_t x2 = lane < 62 ? n2 : lane == 62 ? t0 : t1;
    const uint32_t x3 = lane < 61 ? n3 : lane == 61 ? t0 : lane == 62 ? t1 : t2;
    uint32_t hdr = 0;   // positions whose header fields pass
    uint32_t surv = 0;  // positions passing the whole cheap stage
    if (W < W1) {
      // only candidates in [lo_bit, hi_bit); a dynamic header's 17 bits lie
      // inside the file
      const int64_t b0 = 32 * W - mb;
      const uint32_t keep = bits_in(b0, (int64_t)cd.lo_bit, (int64_t)cd.hi_bit);
      hdr = stage1_header_mask(x0, x1) & keep & bits_in(b0, 0, (int64_t)s.end_bits - 16);
      if (mode & FD_STORED_STARTS) surv = stage1_stored_mask(s, W, x0, x1, x2, x3) & keep;
    }
    // the header survivors of the wave in bit order (lane by lane, bits in a
    // lane ascending): entry lane << 5 | bit, in this wave's table space,
    // which is free until the survivors are checked below
    {
      const uint32_t cnt = (uint32_t)__builtin_popcount(hdr);
      uint32_t at = 0, total = 0;
      for (int bb = 0; bb < 4; bb++) {  // counts are at most 11
        const uint64_t m = __ballot((cnt >> bb) & 1u);
        at += (uint32_t)__builtin_popcountll(m & lanes_below()) << bb;
        total += (uint32_t)__builtin_popcountll(m) << bb;
      }
      uint16_t *list = reinterpret_cast<uint16_t *>(cltab[wave]);
      for (uint32_t p = hdr; p; p &= p - 1) list[at++] = (uint16_t)(((uint32_t)lane << 5) | (uint32_t)__builtin_ctz(p));
      wave_sync();
      for (uint32_t r = 0; r < total; r += 64) {
        const uint32_t i = r + (uint32_t)lane;
        const uint32_t e = i < total ? (uint32_t)list[i] : 0u;
        const int src = (int)(e >> 5);
        const uint32_t y0 = (uint32_t)__shfl((int)x0, src), y1 = (uint32_t)__shfl((int)x1, src);
        const uint32_t y2 = (uint32_t)__shfl((int)x2, src), y3 = (uint32_t)__shfl((int)x3, src);
        const bool ok = i < total && stage1_kraft_ok(y0, y1, y2, y3, e & 31u, k3);
        // survivors are rare: each goes back to its lane's mask
        for (uint64_t m = __ballot(ok); m; m &= m - 1) {
          const uint32_t el = (uint32_t)__builtin_amdgcn_readlane((int)e, __ffsll((unsigned long long)m) - 1);
          if ((uint32_t)lane == (el >> 5)) surv |= 1u << (el & 31u);
        }
      }
      wave_sync();
    }
    // queue the survivors in bit order (lanes in order, bits within a lane)
    uint64_t m = __ballot(surv != 0);
    for (int r = 0; r < 64 && m && !found; r++) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)surv, l);
      for (int x = 0; x < 32 && sl && !found; x++) {
        const uint32_t k = (uint32_t)__builtin_ctz(sl);
        sl &= sl - 1;
        if (lane == 0) q[nq] = (unsigned long long)((uint64_t)(32 * (Wt + l) - mb) + k);
        nq++;
        if (nq == 2 * SCAN_BATCH) found = check(SCAN_BATCH);
      }
    }
    if (!found && nq >= SCAN_BATCH) found = check(SCAN_BATCH);
  }
  // the rest of the queue (all before any step not taken)
  for (int r = 0; r < 4 && !found && nq; r++) found = check(nq < SCAN_BATCH ? nq : SCAN_BATCH);
}

// ---------------------------------------------------------------------------
// k_capacity: one workgroup per file.  A chunk decodes from its start to the
// next chunk start found by the scan, so its symbol capacity is sized from
// that span: factor * span bytes + slack, rounded to the flush unit.  When
// that candidate fails its trial block it may lie inside a block, and the
// chunk decodes to the end of that block, so the span counts at least half
// the chunk's own compressed range (blocks are far shorter than that at the
// default chunk sizes).  The spans partition the payload, so the file's pool
// of factor * (1.5 P + 2 N) + N * (slack + unit) symbols always suffices.
// ---------------------------------------------------------------------------

constexpr int CAP_THREADS = 1024;

__global__ __launch_bounds__(CAP_THREADS) void k_capacity(const FileDesc *files, ChunkDesc *chunks, const ChunkState *cs,
                                                  uint32_t factor) {
  __shared__ uint64_t part[CAP_THREADS];
  __shared__ uint64_t nxt[CAP_THREADS];
  const uint32_t f = blockIdx.x;
  const FileDesc fd = files[f];
  const uint32_t c0 = fd.first_chunk, n = fd.n_chunks;
  const int tid = (int)threadIdx.x;
  // the last chunk decodes to the final block, or past a segment's stop to
  // the end of the block holding it
  const uint64_t tr_bit = 8ull * fd.trailer_byte;
  const uint64_t end_bit = fd.stop_bit == NONE ? tr_bit
                           : fd.stop_bit + 8 * STOP_MARGIN_BYTES < tr_bit ? fd.stop_bit + 8 * STOP_MARGIN_BYTES
                                                                         : tr_bit;
  // pass 1, last tile first: next start after each chunk (suffix minimum)
  uint64_t later = end_bit;
  const uint32_t ntiles = (n + CAP_THREADS - 1) / CAP_THREADS;
  for (uint32_t t = ntiles; t-- > 0;) {
    const uint32_t i = t * CAP_THREADS + (uint32_t)tid;
    uint64_t s = NONE;
    if (i < n) s = (chunks[c0 + i].flags & CF_FIRST) ? fd.payload_bit : cs[c0 + i].cand;
    part[tid] = s;
    __syncthreads();
    // inclusive suffix minimum within the tile
    for (int o = 1; o < CAP_THREADS; o <<= 1) {
      const uint64_t b = tid + o < CAP_THREADS ? part[tid + o] : NONE;
      __syncthreads();
      part[tid] = part[tid] < b ? part[tid] : b;
      __syncthreads();
    }
    const uint64_t after = tid + 1 < CAP_THREADS ? part[tid + 1] : NONE;
    nxt[tid] = after < later ? after : later;
    const uint64_t tile_min = part[0];
    __syncthreads();
    if (i < n) {
      uint64_t cap = 0;
      if (s != NONE && s < end_bit) {
        const uint64_t e = nxt[tid] < end_bit ? nxt[tid] : end_bit;
        // a probe's one block: at most the stop margin of compressed bytes
        const ChunkDesc &cd = chunks[c0 + i];
        const uint64_t half = (cd.hi_bit - cd.lo_bit + 15) / 16;
        const uint64_t to_next = e > s ? (e - s + 7) / 8 : 1;
        const uint64_t span = (fd.mode & FD_PROBE) ? STOP_MARGIN_BYTES : to_next > half ? to_next : half;
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
    const uint32_t i = t * CAP_THREADS + (uint32_t)tid;
    const uint64_t cap = i < n ? chunks[c0 + i].sym_cap : 0;
    part[tid] = cap;
    __syncthreads();
    for (int o = 1; o < CAP_THREADS; o <<= 1) {
      const uint64_t a = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      __syncthreads();
    }
    if (i < n) chunks[c0 + i].sym_off = carry + part[tid] - cap;
    carry += part[CAP_THREADS - 1];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_inflate: persistent; each wave pops chunk indices from the work queue.
// ---------------------------------------------------------------------------

// The 512-symbol ring: at most 96 VGPRs (5 waves per SIMD), so that 18
// decoders fit in a CU's LDS and registers; what does not fit in 96 is
// loop-invariant and reloaded once per chunk.
template <int WIN, bool STORED>
__global__ __launch_bounds__(64, WIN == 512 ? 5 : 1) void k_inflate(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                                const uint32_t *order, uint32_t n, Counters *ctr, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  for (uint32_t it = 0; it <= n; it++) {
    uint32_t item = 0;
    if (lane_id() == 0) item = atomicAdd(&ctr->inflate_next, 1u);
    item = uni(item);
    if (item >= n) break;
    inflate_chunk<WIN, STORED>(sh, files, chunks, cs, pool, order[item], true, NONE);
  }
}

// Passes where few chunks have work: a wave takes 64 chunks per atomic,
// tests them with one lane each, then works on the ones that need it one
// after another (a single shared counter per chunk would serialise).
template <typename Need, typename Work>
__device__ __forceinline__ void sparse_chunks(uint32_t *counter, uint32_t n, Need need, Work work) {
  const int lane = lane_id();
  for (uint32_t it = 0; it <= n / 64u + 1u; it++) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(counter, 64u);
    base = uni(base);
    if (base >= n) break;
    const uint32_t c = base + (uint32_t)lane;
    uint64_t m = __ballot(c < n && need(c));
    for (int q = 0; q < 64 && m; q++) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      work(base + (uint32_t)l);
    }
  }
}

// ---------------------------------------------------------------------------
// k_confirm: a chunk that reached its stop before its trial block and 5
// confirmation blocks were all decoded (Appendix A) still owes the rest,
// which are the blocks after its end.  When the next accepted chunk starts
// exactly there and decoded them with the same checks, they are confirmed
// (its first blocks are checked as its own trial and confirmation; the
// trial's rules are stricter, and nothing checked depends on the history
// before the blocks); the chain is followed while it keeps starting where the
// last one ended.  Otherwise the owed blocks are decoded on their own,
// parsed only.  A failure marks the chunk for k_redo.  Reads only what
// k_inflate wrote (plus its own flag).
// ---------------------------------------------------------------------------

template <int WIN>
__global__ __launch_bounds__(64) void k_confirm(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                                uint32_t n, Counters *ctr, uint16_t *pool, uint32_t always_decode) {
  __shared__ InflateLDS<WIN> sh;
  auto owes = [&](uint32_t c) { return cs[c].pad != 0 && cs[c].start != NONE && cs[c].status == ST_OK; };
  sparse_chunks(&ctr->confirm_next, n, owes, [&](uint32_t c) {
    const uint32_t need0 = uni(cs[c].pad);
    const ChunkDesc cd = chunks[c];
    const FileDesc fd = files[cd.file];
    const uint32_t c1 = fd.first_chunk + fd.n_chunks;
    uint32_t need = need0;
    uint64_t at = uni64(cs[c].end);
    uint32_t x = c;
    bool ok = false;
    for (uint32_t g = 0; g < fd.n_chunks && !ok && !always_decode; g++) {
      uint32_t xn = x + 1;
      for (uint32_t h = 0; h < fd.n_chunks && xn < c1 && uni64(cs[xn].start) == NONE; h++) xn++;
      // the chain reached a segment's stop: the blocks still owed are the
      // next segment's first ones, decoded from this proven end; the start
      // itself is proven or repaired by the chain check of k_finalize
      if (xn >= c1 && fd.stop_bit != NONE && at >= fd.stop_bit) {
        ok = true;
        break;
      }
      if (xn >= c1 || uni64(cs[xn].start) != at || uni(cs[xn].status) != ST_OK) break;
      const uint32_t kx = uni(cs[xn].n_blocks);
      if ((uni(cs[xn].flags) & CS_FINAL) || kx >= need) {
        ok = true;
        break;
      }
      need -= kx;
      at = uni64(cs[xn].end);
      x = xn;
    }
    if (!ok) {
      Inflater<WIN> inf(sh);
      inflater_setup(inf, fd, cd, pool);
      ok = inf.confirm(at, need) == D_OK;
    }
    if (!ok && lane_id() == 0) cs[c].flags |= CS_UNCONFIRMED;
  });
}

// k_redo: a chunk whose candidate failed its deferred confirmation searches
// the next candidate and decodes it with the whole confirmation.
template <int WIN>
__global__ __launch_bounds__(64) void k_redo(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs, uint32_t n,
                                             Counters *ctr, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  auto rejected = [&](uint32_t c) { return (cs[c].flags & CS_UNCONFIRMED) != 0; };
  sparse_chunks(&ctr->redo_next, n, rejected, [&](uint32_t c) {
    const uint64_t s0 = uni64(cs[c].start);
    const uint32_t r0 = uni(cs[c].retries);
    inflate_chunk<WIN, true>(sh, files, chunks, cs, pool, c, false, s0 + 1);
    if (lane_id() == 0) {
      cs[c].retries += r0 + 1;
      cs[c].confirm_rej += 1;
    }
  });
}

// Symbols that chunk c may hold once the accepted starts are final: its own
// region and those of the empty chunks after it, up to the region of `next`,
// the next chunk with a start (pool regions lie in chunk order, back to
// back).  A candidate rejected after the regions were sized leaves its chunk
// empty, and the chunk before it decodes on through that chunk's range.
__device__ __forceinline__ uint64_t region_to_next(const FileDesc &fd, const ChunkDesc *chunks, uint32_t c,
                                                   uint32_t next) {
  const uint64_t end = next < fd.first_chunk + fd.n_chunks ? chunks[next].sym_off : fd.pool_base + fd.pool_elems;
  return end > chunks[c].sym_off ? end - chunks[c].sym_off : 0;
}

// Continue chunk c from its recorded end (a cut chunk: from the last block
// boundary whose symbols were stored) until the first block at or past
// `stop`, with room for `cap` symbols.
template <int WIN>
__device__ void extend_chunk(InflateLDS<WIN> &sh, const FileDesc &fd, const ChunkDesc &cd, ChunkState *cs,
                             uint16_t *pool, uint32_t c, uint64_t stop, uint64_t cap) {
  const int lane = lane_id();
  Inflater<WIN> inf(sh);
  inflater_setup(inf, fd, cd, pool);
  inf.cap = cap;
  const bool cut = (uni(cs[c].flags) & CS_CUT) != 0;
  const uint64_t len = uni64(cs[c].len);
  const uint64_t e = cut ? uni64(cs[c].cut_bit) : uni64(cs[c].end);
  const uint32_t nb0 = cut ? uni(cs[c].cut_blocks) : uni(cs[c].n_blocks);
  // bring the recent history back into the ring
  const uint64_t h0 = len > (uint64_t)WIN ? len - WIN : 0;
  for (uint64_t p = h0 + (uint64_t)lane; p < len; p += 64)
    sh.ring[p & (WIN - 1)] = p < cap ? inf.D[p] : (uint16_t)0;
  wave_sync();
  inf.pos = len;
  inf.flushed = len & ~(uint64_t)(Inflater<WIN>::UNIT - 1);
  DecodeResult r = inf.run(e, stop, 0u);
  uint32_t ph = wave_sum(inf.nph_stop);
  if (lane == 0) {
    bool overflow = inf.over && r.len > cap;
    cs[c].end = r.end;
    cs[c].len = r.len;
    cs[c].n_blocks = nb0 + r.blocks;
    cs[c].n_syms += inf.nsyms;
    cs[c].n_placeholders += ph;
    cs[c].flags = (cs[c].flags & ~CS_FINAL) | CS_EXTENDED | (r.final_seen ? CS_FINAL : 0u) |
                  (overflow ? CS_OVERFLOW : 0u);
    if (r.status != D_OK) cs[c].status = ST_DATA;
    else if (overflow) {
      cs[c].status = ST_CAPACITY;
      cs[c].needed = r.len;
    }
  }
}

// Decode chunk c again from `start` with a placeholder context (repair),
// with room for `cap` symbols.
template <int WIN>
__device__ void redecode_chunk(InflateLDS<WIN> &sh, const FileDesc &fd, const ChunkDesc &cd, ChunkState *cs,
                               uint16_t *pool, uint32_t c, uint64_t start, uint64_t stop, uint64_t cap) {
  const int lane = lane_id();
  Inflater<WIN> inf(sh);
  inflater_setup(inf, fd, cd, pool);
  inf.cap = cap;
  DecodeResult r = inf.run(start, stop, 0u);
  uint32_t ph = wave_sum(inf.nph_stop);
  if (lane == 0) {
    bool overflow = inf.over && r.len > cap;
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
// chunks are empty), continue to it.  A chunk that outgrew its capacity in
// pass 1 (CS_CUT) continues from its last stored block boundary, with the
// room of the empty chunks after it.
// ---------------------------------------------------------------------------

template <int WIN>
__global__ __launch_bounds__(64) void k_stitch(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                               uint32_t n, Counters *ctr, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  // a chunk continues when the next accepted start lies past its end
  auto short_of_next = [&](uint32_t c) {
    if (cs[c].start == NONE || cs[c].status != ST_OK) return false;
    if (cs[c].flags & CS_CUT) return true;  // pass 1 stored only part of it
    if (cs[c].flags & CS_FINAL) return false;
    const FileDesc &fd = files[chunks[c].file];
    const uint64_t nf = next_start(fd, cs, c, true, nullptr);
    return cs[c].end < nf || nf == NONE;
  };
  sparse_chunks(&ctr->stitch_next, n, short_of_next, [&](uint32_t c) {
    const ChunkDesc cd = chunks[c];
    const FileDesc fd = files[cd.file];
    uint32_t nx;
    const uint64_t nf = uni64(next_start(fd, cs, c, true, &nx));
    extend_chunk<WIN>(sh, fd, cd, cs, pool, c, nf, region_to_next(fd, chunks, c, uni(nx)));
  });
}

// ---------------------------------------------------------------------------
// k_finalize: one workgroup per file.  Checks that every accepted start is
// the previous chunk's end, repairs sequentially if not, then the exclusive
// scan of the chunk lengths gives the output offsets.  A chunk that starts
// on a stored header at s after a chunk that ended at e, s < e, in the same
// run of zero bits before the same LEN/NLEN, began the same block: its start
// becomes e with nothing decoded again.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool stored_equivalent(const FileDesc &fd, uint64_t s, uint64_t e) {
  if (!(fd.mode & FD_STORED_STARTS) || !(s < e) || ((s + 10u) >> 3) != ((e + 10u) >> 3)) return false;
  Src src;
  src.init(fd.comp, fd.comp_len);
  const uint64_t v = src.peek64(s);
  return (v & 7u) == 0u && stored_start_bits(v, s, src.end_bits);
}

constexpr int FIN_THREADS = 1024;

template <int WIN>
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                                                  FileState *fs, uint16_t *pool) {
  __shared__ InflateLDS<WIN> sh;
  __shared__ int bad;
  __shared__ uint64_t part[FIN_THREADS];
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
    if (sp.status == ST_OK && !(sp.flags & CS_FINAL) && sp.end != sj.start && stored_equivalent(fd, sj.start, sp.end)) {
      cs[j].start = sp.end;  // the same stored block: the same symbols and end
      continue;
    }
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
      if (j != c0 && sj != cur && stored_equivalent(fd, sj, cur)) {
        if (tid == 0) cs[j].start = cur;
      } else if (j != c0 && sj != cur) {
        repairs++;
        uint32_t nx;
        uint64_t stop = uni64(next_start(fd, cs, j, true, &nx));
        if (cur >= stop) {
          // the previous chunk already decoded through this one's range:
          // nothing of its own decode from the false start is kept
          if (tid == 0) {
            cs[j].start = cur;
            cs[j].end = cur;
            cs[j].len = 0;
            cs[j].n_blocks = 0;
            cs[j].n_syms = 0;
            cs[j].n_placeholders = 0;
            cs[j].flags = CS_REPAIRED;
            cs[j].status = ST_OK;
          }
        } else {
          redecode_chunk<WIN>(sh, fd, chunks[j], cs, pool, j, cur, stop, region_to_next(fd, chunks, j, uni(nx)));
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
    if (st == ST_OK && !fin && fd.stop_bit == NONE) st = ST_DATA;  // stream ends without a final block
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
    // Hillis-Steele inclusive scan (FIN_THREADS entries)
    for (int o = 1; o < FIN_THREADS; o <<= 1) {
      uint64_t a = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      __syncthreads();
    }
    if (j < c1) {
      const uint64_t off = carry + part[tid] - L;
      cs[j].out_off = off;
      const uint64_t hist = off + fd.win_valid;
      cs[j].valid = (uint32_t)(hist < WINDOW ? hist : WINDOW);
    }
    carry += part[FIN_THREADS - 1];
    __syncthreads();
  }
  // reductions of the statistics
  part[tid] = nsyms;
  __syncthreads();
  for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_syms = part[0];
  __syncthreads();
  part[tid] = nph;
  __syncthreads();
  for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_ph = part[0];
  __syncthreads();
  part[tid] = nblk | ((uint64_t)nonempty << 40);
  __syncthreads();
  for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  const uint64_t tot_blk = part[0] & ((1ull << 40) - 1), tot_ne = part[0] >> 40;
  __syncthreads();
  part[tid] = (uint64_t)ext | ((uint64_t)retries << 20) | ((uint64_t)overflow << 42);
  __syncthreads();
  for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
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
    const bool fin = (last_flags & CS_FINAL) != 0;
    // the member's trailer: the last 8 bytes, or (when more members may
    // follow) the 8 bytes from the byte boundary after the final block
    const bool members = (fd.mode & FD_MEMBERS) != 0;
    const uint64_t tr = fin ? ((last_end + 7) >> 3) : 0;
    uint32_t tcrc = fd.crc, tisize = fd.isize;
    if (st == ST_OK) {
      // a segment stops at a block boundary past its stop, or ends the member
      if (!fin && (fd.stop_bit == NONE || last_end == NONE || last_end < fd.stop_bit)) st = ST_DATA;
      else if (fin && !members && tr + 8 != fd.comp_len) st = ST_UNSUPPORTED;
      else if (fin && members && tr + 8 > fd.comp_len) st = ST_DATA;  // truncated trailer
      else if (ovf) st = ST_CAPACITY;
      else if (carry > fd.out_cap) st = ST_CAPACITY;
    }
    if (fin && members && tr + 8 <= fd.comp_len) {
      tcrc = tisize = 0;
      for (int k = 3; k >= 0; k--) {
        tcrc = (tcrc << 8) | fd.comp[tr + k];
        tisize = (tisize << 8) | fd.comp[tr + 4 + k];
      }
    }
    fs[f].trailer_crc = tcrc;
    fs[f].trailer_isize = tisize;
    // a length that differs from ISIZE is reported after the CRC check
    fs[f].size_bad = fin && (uint32_t)(fd.out_before + carry) != tisize ? 1u : 0u;
    fs[f].is_final = fin ? 1u : 0u;
    fs[f].end_bit = last_end;
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
// Window propagation (pass 2a).  The window of the next accepted chunk is
// w_next[k] = t < 256 ? t : w[t & 0x7FFF], t = symbol k of the last 32768 of
// (w_hat_i ++ D_i); a file's first chunk has no history (its window, unused,
// is zero), except the first chunk of a segment of a longer member, whose
// window (the bytes before the segment) the host placed in its slot of
// `wins`.  The chain over all accepted chunks (the compacted list of the
// size scan, files one after another) is cut into segments of PSEG chunks:
//   k_prop_maps   each segment composes its steps into one map from its input
//                 window to the next segment's (16-bit entries: a byte, or
//                 0x8000 | position in the input window), all segments at once
//   k_prop_scan   prefix compositions of the maps, log2(S) rounds over all
//                 segments at once (composition is associative: (A o B)[k]
//                 is A[k] if a byte, else B[A[k] & 0x7FFF])
//   k_prop_segwin every segment's input window: its prefix map applied to
//                 the first window
//   k_prop_apply  each segment runs its steps from its input window and
//                 stores every chunk's window
// so nothing is sequential over segments: the chain of S steps is a scan.
// Each step: every thread gathers 32 of the 32768 entries into registers,
// then (after a barrier) writes them; the next chunk's tail is loaded while
// the current one is resolved.
// ---------------------------------------------------------------------------

constexpr int PROP_THREADS = 1024;
constexpr int PROP_PER = WINDOW / PROP_THREADS;
constexpr uint32_t PSEG = 64;

// symbols k = i * PROP_THREADS + tid of the last 32768 of (w_hat ++ D_j),
// two 16-bit symbols per register (i even: low half)
__device__ __forceinline__ void load_tail(const uint16_t *__restrict__ Dj, uint64_t L, int tid,
                                          uint32_t (&t)[PROP_PER / 2]) {
#pragma unroll
  for (int i = 0; i < PROP_PER; i++) {
    const uint64_t q = L + (uint64_t)(i * PROP_THREADS + tid);
    const uint32_t x = q < WINDOW ? (0x8000u | (uint32_t)q) : (uint32_t)Dj[q - WINDOW];
    if (i & 1) t[i >> 1] |= x << 16;
    else t[i >> 1] = x;
  }
}

// One segment's steps over list positions q0 .. q1 - 1: T is uint16_t for
// maps (k_prop_maps, `to_end`: the last step gives the window of position q1,
// the next segment's first) or uint8_t for windows (k_prop_apply: windows of
// q0 (store_first) .. q1 - 1 go to `wins`; position q1 may not exist).  `buf`
// holds the window of position q0 on entry.  A carried window is read from
// its slot in `seed` (slots that are never written here).
template <typename T>
__device__ __forceinline__ void prop_steps(T *buf, const AccEntry *acc, const uint16_t *__restrict__ pool, uint32_t q0,
                                           uint32_t q1, const uint8_t *seed, uint8_t *wins, bool store_first,
                                           bool to_end) {
  const int tid = (int)threadIdx.x;
  uint32_t t[PROP_PER / 2], tn[PROP_PER / 2];
  AccEntry e0 = acc[q0];
  if (store_first && wins && !(e0.pad & 1u)) {
    uint8_t *wo = wins + (uint64_t)e0.chunk * WINDOW;
    for (int k = tid; k < (int)WINDOW; k += PROP_THREADS) wo[k] = (uint8_t)buf[k];
  }
  load_tail(pool + e0.sym_off, e0.len, tid, t);
  AccEntry e1 = q0 + 1 < q1 ? acc[q0 + 1] : e0;
  const uint32_t qend = to_end ? q1 : q1 - 1;
  for (uint32_t q = q0; q < qend; q++) {
    // window of position q + 1 from the tail of q (the next tail is loaded meanwhile)
    const bool have_next = q + 1 < q1;
    AccEntry e2 = e1;
    if (have_next) {
      if (q + 2 < q1) e2 = acc[q + 2];
      load_tail(pool + e1.sym_off, e1.len, tid, tn);
    }
    // a file's first chunk starts without history, or from its carried window
    const AccEntry en = q + 1 < q1 ? e1 : acc[q + 1];
    const bool reset = en.pad & 1u;
    const uint8_t *carried = (en.pad & 2u) ? seed + (uint64_t)en.chunk * WINDOW : nullptr;
    uint32_t v[PROP_PER / 2];  // two results per register
#pragma unroll
    for (int i = 0; i < PROP_PER; i++) {
      const uint32_t x = (t[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
      uint32_t y = x < 256u ? x : (uint32_t)buf[x & 0x7FFFu];
      if (reset) y = carried ? (uint32_t)carried[i * PROP_THREADS + tid] : 0u;
      if (i & 1) v[i >> 1] |= y << 16;
      else v[i >> 1] = y;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PROP_PER; i++) buf[i * PROP_THREADS + tid] = (T)(v[i >> 1] >> (16 * (i & 1)));
    if (wins && have_next && !reset) {
      uint8_t *wo = wins + (uint64_t)e1.chunk * WINDOW;
#pragma unroll
      for (int i = 0; i < PROP_PER; i++) wo[i * PROP_THREADS + tid] = (uint8_t)(v[i >> 1] >> (16 * (i & 1)));
    }
    __syncthreads();
    e1 = e2;
#pragma unroll
    for (int i = 0; i < PROP_PER / 2; i++) t[i] = tn[i];
  }
}

__global__ __launch_bounds__(PROP_THREADS) void k_prop_maps(const uint32_t *acc_pos, uint32_t n, const AccEntry *acc,
                                                            const uint16_t *__restrict__ pool, const uint8_t *seed,
                                                            uint16_t *maps) {
  __shared__ uint16_t m[WINDOW];
  const uint32_t A = acc_pos[n], g = blockIdx.x;
  const uint32_t q0 = g * PSEG;
  if (q0 + PSEG >= A) return;  // the last segment has no successor
  for (int k = threadIdx.x; k < (int)WINDOW; k += PROP_THREADS) m[k] = (uint16_t)(0x8000u | (uint32_t)k);
  __syncthreads();
  // map from the window of q0 to the window of q0 + PSEG
  prop_steps<uint16_t>(m, acc, pool, q0, q0 + PSEG, seed, nullptr, false, true);
  uint16_t *mo = maps + (uint64_t)g * WINDOW;
  for (int k = threadIdx.x; k < (int)WINDOW; k += PROP_THREADS) mo[k] = m[k];
}

// One round of the prefix composition: out[g] = in[g] o in[g - dist] for
// g >= dist, else in[g] (maps exist for segments 0 .. S - 2).  Grid:
// PROP_PARTS blocks per segment, each over a part of the 32768 entries.
constexpr uint32_t PROP_PARTS = 32;
__global__ __launch_bounds__(256) void k_prop_scan(const uint32_t *acc_pos, uint32_t n,
                                                   const uint16_t *__restrict__ in, uint16_t *__restrict__ out,
                                                   uint32_t dist) {
  const uint32_t A = acc_pos[n];
  const uint32_t S = (A + PSEG - 1) / PSEG;
  const uint32_t g = blockIdx.x / PROP_PARTS, part = blockIdx.x % PROP_PARTS;
  if (g + 1 >= S) return;
  const uint16_t *mg = in + (uint64_t)g * WINDOW;
  const uint16_t *mp = g >= dist ? in + (uint64_t)(g - dist) * WINDOW : nullptr;
  uint16_t *og = out + (uint64_t)g * WINDOW;
  for (uint32_t k = part * blockDim.x + threadIdx.x; k < WINDOW; k += PROP_PARTS * blockDim.x) {
    uint32_t x = mg[k];
    if (mp && x >= 256u) x = mp[x & 0x7FFFu];
    og[k] = (uint16_t)x;
  }
}

// Segment g's input window: the first window (carried in, or none) for
// g = 0, else the prefix map of segments 0 .. g - 1 applied to it.
__global__ __launch_bounds__(256) void k_prop_segwin(const uint32_t *acc_pos, uint32_t n, const AccEntry *acc,
                                                     const uint16_t *__restrict__ prefix, const uint8_t *seed,
                                                     uint8_t *__restrict__ segwin) {
  const uint32_t A = acc_pos[n];
  const uint32_t S = (A + PSEG - 1) / PSEG;
  const uint32_t g = blockIdx.x / PROP_PARTS, part = blockIdx.x % PROP_PARTS;
  if (g >= S) return;
  const uint8_t *w0 = A > 0 && (acc[0].pad & 2u) ? seed + (uint64_t)acc[0].chunk * WINDOW : nullptr;
  const uint16_t *pg = g > 0 ? prefix + (uint64_t)(g - 1) * WINDOW : nullptr;
  uint8_t *wo = segwin + (uint64_t)g * WINDOW;
  for (uint32_t k = part * blockDim.x + threadIdx.x; k < WINDOW; k += PROP_PARTS * blockDim.x) {
    uint32_t x = pg ? (uint32_t)pg[k] : 0x8000u | k;
    if (x >= 256u) x = w0 ? w0[x & 0x7FFFu] : 0u;
    wo[k] = (uint8_t)x;
  }
}

__global__ __launch_bounds__(PROP_THREADS) void k_prop_apply(const uint32_t *acc_pos, uint32_t n, const AccEntry *acc,
                                                             const uint16_t *__restrict__ pool,
                                                             const uint8_t *__restrict__ segwin,
                                                             uint8_t *__restrict__ wins) {
  __shared__ uint8_t w[WINDOW];
  const uint32_t A = acc_pos[n], g = blockIdx.x;
  const uint32_t q0 = g * PSEG;
  if (q0 >= A) return;
  const uint8_t *wi = segwin + (uint64_t)g * WINDOW;
  for (int k = threadIdx.x; k < (int)WINDOW; k += PROP_THREADS) w[k] = wi[k];
  __syncthreads();
  prop_steps<uint8_t>(w, acc, pool, q0, min(q0 + PSEG, A), wins, wins, true, false);
}

// ---------------------------------------------------------------------------
// k_tilescan: one workgroup; tiles[j] = translate tiles before chunk j over
// the whole batch (files whose status is not OK contribute none).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tilescan(const ChunkDesc *chunks, const ChunkState *cs, const FileState *fs,
                                                   uint32_t n, uint64_t *tiles, uint32_t *acc_pos, AccEntry *acc) {
  __shared__ uint64_t part[1024];
  __shared__ uint32_t apart[1024];
  const int tid = (int)threadIdx.x;
  uint64_t carry = 0;
  uint32_t acarry = 0;
  for (uint32_t base = 0; base < n; base += 1024) {
    const uint32_t j = base + (uint32_t)tid;
    uint64_t T = 0;
    uint32_t A = 0;
    if (j < n && cs[j].start != NONE) {
      A = 1;
      if (fs[chunks[j].file].status == ST_OK) T = (cs[j].len + TRANSLATE_TILE - 1) / TRANSLATE_TILE;
    }
    part[tid] = T;
    apart[tid] = A;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      uint64_t a = tid >= o ? part[tid - o] : 0;
      uint32_t b = tid >= o ? apart[tid - o] : 0;
      __syncthreads();
      part[tid] += a;
      apart[tid] += b;
      __syncthreads();
    }
    if (j < n) {
      tiles[j] = carry + part[tid] - T;
      const uint32_t ap = acarry + apart[tid] - A;
      acc_pos[j] = ap;
      if (A) {
        AccEntry e;
        e.sym_off = chunks[j].sym_off;
        // a file that failed is not translated: its chunks' symbols are not
        // read (their length may exceed what was stored)
        e.len = fs[chunks[j].file].status == ST_OK ? cs[j].len : 0;
        e.chunk = j;
        // the chain restarts at a file's first chunk, from the carried window
        // of a segment or from nothing
        e.pad = ((chunks[j].flags & CF_FIRST) ? 1u : 0u) | ((chunks[j].flags & CF_CARRIED) ? 2u : 0u);
        acc[ap] = e;
      }
    }
    carry += part[1023];
    acarry += apart[1023];
    __syncthreads();
  }
  if (tid == 0) {
    tiles[n] = carry;
    acc_pos[n] = acarry;
  }
}

// ---------------------------------------------------------------------------
// k_translate: out[o_i + p] = D_i[p] < 256 ? D_i[p] : w_i[D_i[p] & 0x7FFF].
// A persistent grid pulls whole chunks: the chunk's window goes to LDS once
// (when the chunk has placeholders), then the chunk is walked in pieces of
// TRANSLATE_TILE symbols whose placeholders are looked up there.  `tiles`
// (the tile prefix of the size scan) is only used for its total: a batch
// whose files failed translates nothing.
// ---------------------------------------------------------------------------

constexpr uint32_t TRANSLATE_THREADS = 256;
static_assert(TRANSLATE_TILE % (8u * TRANSLATE_THREADS) == 0, "translate piece");

__global__ __launch_bounds__(TRANSLATE_THREADS) void k_translate(const FileDesc *files, const ChunkDesc *chunks, const ChunkState *cs,
                                                   FileState *fs, const uint64_t *tiles, uint32_t n,
                                                   const uint8_t *wins, const uint16_t *pool, Counters *ctr) {
  __shared__ uint32_t s_item;
  __shared__ uint4 wlw[WINDOW / 16];                 // the chunk's window
  __shared__ uint4 tbw[(TRANSLATE_TILE + 32) / 16];  // 16-byte aligned staging
  const uint8_t *wl = reinterpret_cast<const uint8_t *>(wlw);
  uint8_t *tb = reinterpret_cast<uint8_t *>(tbw);
  if (tiles[n] == 0) return;
  for (uint32_t it = 0; it <= n; it++) {
    if (threadIdx.x == 0) s_item = atomicAdd(&ctr->translate_next, 1u);
    __syncthreads();
    const uint32_t j = s_item;
    __syncthreads();
    if (j >= n) break;
    const ChunkState sj = cs[j];
    if (sj.start == NONE || sj.len == 0) continue;
    const uint32_t f = chunks[j].file;
    if (fs[f].status != ST_OK) continue;
    const FileDesc fd = files[f];
    const uint64_t L = sj.len;
    const uint16_t *Dj = pool + chunks[j].sym_off;
    const uint32_t lim = 32768u - sj.valid;  // placeholders below this lie before the data start
    uint8_t *out = fd.out + sj.out_off;
    // (with no history before the chunk every placeholder is a data error,
    // whatever the window holds)
    if (sj.valid) {
      const uint4 *wj = reinterpret_cast<const uint4 *>(wins + (uint64_t)j * WINDOW);
      static_assert(WINDOW % (16u * TRANSLATE_THREADS) == 0, "window load");
      uint4 wv[WINDOW / (16u * TRANSLATE_THREADS)];
#pragma unroll
      for (uint32_t i = 0; i < WINDOW / (16u * TRANSLATE_THREADS); i++) wv[i] = wj[threadIdx.x + TRANSLATE_THREADS * i];
#pragma unroll
      for (uint32_t i = 0; i < WINDOW / (16u * TRANSLATE_THREADS); i++) wlw[threadIdx.x + TRANSLATE_THREADS * i] = wv[i];
      __syncthreads();
    }
    int err = 0;
    for (uint64_t p0 = 0; p0 < L; p0 += TRANSLATE_TILE) {
      // a piece's bytes are staged in LDS at the output's alignment, then
      // stored as aligned 16-byte words (byte stores for the partial words
      // at the two ends, which the neighbouring pieces share)
      const uint64_t cnt = L - p0 < TRANSLATE_TILE ? L - p0 : TRANSLATE_TILE;
      const uintptr_t ob = (uintptr_t)(out + p0);
      const uint32_t sh = (uint32_t)(ob & 15u);
      // all of a thread's loads of the piece are issued before any is used
      constexpr uint32_t PER = TRANSLATE_TILE / (8u * TRANSLATE_THREADS);
      uint4 v[PER];
#pragma unroll
      for (uint32_t i = 0; i < PER; i++) {
        const uint64_t g = p0 + 8ull * (threadIdx.x + TRANSLATE_THREADS * i);
        v[i] = g < p0 + cnt ? *reinterpret_cast<const uint4 *>(Dj + g) : uint4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (uint32_t i = 0; i < PER; i++) {
        const uint64_t g = p0 + 8ull * (threadIdx.x + TRANSLATE_THREADS * i);
        const uint32_t w[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
        for (int h = 0; h < 8; h++) {
          const uint64_t p = g + h;
          if (p < p0 + cnt) {
            const uint32_t t = (w[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
            uint32_t b;
            if (t < 256u) {
              b = t;
            } else {
              const uint32_t m = t & 0x7FFFu;
              if (t < 0x8000u || m < lim) err = 1;
              b = wl[m];
            }
            tb[sh + (p - p0)] = (uint8_t)b;
          }
        }
      }
      __syncthreads();
      const uint32_t end = sh + (uint32_t)cnt;      // LDS bytes [sh, end) hold the piece
      const uint32_t first = (sh + 15u) & ~15u;     // first whole 16-byte word
      const uint32_t last = end & ~15u;             // end of the whole words
      uint8_t *base = (uint8_t *)(ob - sh);         // 16-byte aligned
      if (first <= last) {
        for (uint32_t k = first + 16u * threadIdx.x; k < last; k += 16u * blockDim.x)
          *reinterpret_cast<uint4 *>(base + k) = *reinterpret_cast<const uint4 *>(&tb[k]);
        for (uint32_t k = sh + threadIdx.x; k < first; k += blockDim.x) base[k] = tb[k];
        for (uint32_t k = last + threadIdx.x; k < end; k += blockDim.x) base[k] = tb[k];
      } else {
        for (uint32_t k = sh + threadIdx.x; k < end; k += blockDim.x) base[k] = tb[k];
      }
      __syncthreads();
    }
    if (err) atomicCAS(&fs[f].status, ST_OK, ST_DATA);
  }
}

// ---------------------------------------------------------------------------
// k_crc: CRC-32 of every file's output (RFC 1952 section 8), on the device.
// The CRC register without its preset and final inversion is linear over
// GF(2): for a message cut into pieces, raw(M) is the XOR over the pieces of
// raw(piece) * x^(8 * bytes after the piece) mod P.  Each lane takes 256
// bytes (four table lookups per 4 bytes: the slicing technique with tables
// of a byte followed by 0..3 zero bytes), multiplies its raw CRC by the
// power of x for the bytes after it, and the wave's XOR goes to the file's
// accumulator with one atomic XOR, so units need no order.  k_crc_final adds
// the preset (0xFFFFFFFF * x^(8 L)) and the final inversion, then checks the
// trailer; a length differing from ISIZE is reported only when the CRC
// matches, the order in which RFC 1952 lists the two checks.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t gf_mulx(uint32_t a) { return (a >> 1) ^ (CRC_POLY & (0u - (a & 1u))); }

// a * b mod P, reflected representation (bit 31 is x^0)
__device__ __forceinline__ uint32_t gf_mul(uint32_t a, uint32_t b) {
  uint32_t p = 0;
#pragma unroll
  for (int i = 0; i < 32; i++) {
    p ^= b & (0u - ((a >> (31 - i)) & 1u));
    b = gf_mulx(b);
  }
  return p;
}

// x^(8 n) mod P
__device__ __forceinline__ uint32_t gf_xpow8(uint64_t n, const uint32_t *xpow) {
  uint32_t r = 0x80000000u;
  for (int k = 0; k < CRC_XPOW && (n >> k); k++)
    if ((n >> k) & 1u) r = gf_mul(r, xpow[k]);
  return r;
}

// x^(8 n) mod P for a wave-uniform n: lane k holds the factor of bit k,
// multiplied together in a butterfly (every lane ends with the product)
__device__ __forceinline__ uint32_t gf_xpow8_wave(uint64_t n, const uint32_t *xpow) {
  const int lane = lane_id();
  uint32_t f = (lane < CRC_XPOW && ((n >> lane) & 1u)) ? xpow[lane] : 0x80000000u;
  for (int o = 1; o < 64; o <<= 1) f = gf_mul(f, __shfl_xor(f, o));
  return f;
}

__global__ __launch_bounds__(256) void k_crc(const FileDesc *files, uint32_t n_files, FileState *fs,
                                             const uint32_t *consts, uint64_t total_units) {
  __shared__ uint32_t S[4][256];
  const int tid = (int)threadIdx.x;
  {
    uint32_t r = (uint32_t)tid;
#pragma unroll
    for (int k = 0; k < 8; k++) r = (r >> 1) ^ (CRC_POLY & (0u - (r & 1u)));
    S[0][tid] = r;
  }
  __syncthreads();
  for (int k = 1; k < 4; k++) {
    const uint32_t p = S[k - 1][tid];
    S[k][tid] = (p >> 8) ^ S[0][p & 0xFFu];
    __syncthreads();
  }
  const uint64_t unit = (uint64_t)blockIdx.x * 4u + (uint64_t)uni32((uint32_t)tid >> 6);
  if (unit >= total_units) return;
  // file: the last one whose first unit is at or before this one
  uint32_t lo = 0, hi = n_files;
  for (int it = 0; it < 32 && hi - lo > 1; it++) {
    const uint32_t mid = (lo + hi) >> 1;
    if (files[mid].crc_unit0 <= unit) lo = mid;
    else hi = mid;
  }
  const uint32_t f = uni32(lo);
  if (uni(fs[f].status) != ST_OK) return;
  const uint64_t L = uni64(fs[f].out_len);
  const uint64_t start = (unit - files[f].crc_unit0) * CRC_UNIT;
  if (start >= L) return;
  const uint8_t *out = files[f].out;
  const int lane = lane_id();
  const uint64_t a = start + (uint64_t)lane * CRC_LANE;
  const uint64_t b = a + CRC_LANE < L ? a + CRC_LANE : L;
  uint32_t r = 0;
  uint64_t p = a;
  if (((uintptr_t)out & 15u) == 0) {
    // a whole 128-byte line per lane per step, loaded before it is folded in
    // (lanes are CRC_LANE bytes apart, so each line is fetched once)
    for (; p + 128 <= b; p += 128) {
      uint4 q[8];
#pragma unroll
      for (int u = 0; u < 8; u++) q[u] = *reinterpret_cast<const uint4 *>(out + p + 16 * u);
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const uint32_t w4[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
#pragma unroll
        for (int h = 0; h < 4; h++) {
          const uint32_t w = r ^ w4[h];
          r = S[3][w & 0xFFu] ^ S[2][(w >> 8) & 0xFFu] ^ S[1][(w >> 16) & 0xFFu] ^ S[0][w >> 24];
        }
      }
    }
    for (; p + 16 <= b; p += 16) {
      const uint4 q = *reinterpret_cast<const uint4 *>(out + p);
      const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int h = 0; h < 4; h++) {
        const uint32_t w = r ^ w4[h];
        r = S[3][w & 0xFFu] ^ S[2][(w >> 8) & 0xFFu] ^ S[1][(w >> 16) & 0xFFu] ^ S[0][w >> 24];
      }
    }
  }
  for (; p < b; p++) r = S[0][(r ^ out[p]) & 0xFFu] ^ (r >> 8);
  uint32_t v;
  if (start + CRC_UNIT <= L) {
    // full unit: lane m is followed by (63 - m) lanes of the unit, then the rest of the file
    v = gf_mul(r, consts[CRC_XPOW + 63 - lane]);
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o);
    v = gf_mul(v, gf_xpow8_wave(L - (start + CRC_UNIT), consts));
  } else {
    // the file's last unit: each lane's own distance to the end
    v = a < b ? gf_mul(r, gf_xpow8(L - b, consts)) : 0u;
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o);
  }
  if (lane == 0 && v) atomicXor(&fs[f].crc_acc, v);
}

__global__ __launch_bounds__(256) void k_crc_final(const FileDesc *files, uint32_t n_files, FileState *fs,
                                                   const uint32_t *xpow) {
  for (uint32_t f = threadIdx.x; f < n_files; f += blockDim.x) {
    if (fs[f].status != ST_OK) continue;
    const uint64_t L = fs[f].out_len;
    // the register after the earlier bytes is the complement of their CRC
    // (all ones for none), carried over this segment's L bytes
    const uint32_t crc = fs[f].crc_acc ^ gf_mul(~files[f].crc_in, gf_xpow8(L, xpow)) ^ 0xFFFFFFFFu;
    fs[f].crc_out = crc;
    if (!fs[f].is_final || (files[f].mode & FD_NOCHECK)) continue;
    if (crc != fs[f].trailer_crc) fs[f].status = ST_CRC;
    else if (fs[f].size_bad) fs[f].status = ST_SIZE;
  }
}

// ---------------------------------------------------------------------------
// k_carry: the window after a segment (bounded-memory streaming): the last
// 32768 bytes of (the carried window ++ the segment's output), bytes before
// the member's start as zero.  One workgroup; `dst` is not the carried slot.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_carry(const FileDesc *files, const FileState *fs, const uint8_t *wins,
                                                uint8_t *__restrict__ dst) {
  const FileDesc fd = files[0];
  if (fs[0].status != ST_OK) return;
  const int64_t L = (int64_t)fs[0].out_len;
  const uint8_t *old = wins + (uint64_t)fd.first_chunk * WINDOW;
  const int64_t lim = (int64_t)WINDOW - (int64_t)fd.win_valid;
  for (int k = threadIdx.x; k < (int)WINDOW; k += blockDim.x) {
    const int64_t pos = L - (int64_t)WINDOW + k;  // position in the segment's output
    uint8_t b = 0;
    if (pos >= 0) b = fd.out[pos];
    else if ((int64_t)WINDOW + pos >= lim) b = old[WINDOW + pos];
    dst[k] = b;
  }
}

// ---------------------------------------------------------------------------
// k_count_byte: counts[(first + i) / window] += (buf[i] == value), i < n;
// windows past n_counts are not counted.  Each thread takes 16 aligned bytes
// of the global position space per step; a thread's per-window total is added
// once per window it touches.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_count_byte(const uint8_t *__restrict__ buf, uint64_t n, uint32_t value,
                                                    uint64_t first, uint64_t window, unsigned long long *counts,
                                                    uint64_t n_counts) {
  const uint64_t stride = 16ull * gridDim.x * blockDim.x;
  uint64_t cur_w = NONE;
  unsigned long long acc = 0;
  for (uint64_t g = 16ull * (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x); g < n; g += stride) {
    const uint32_t lim = n - g < 16 ? (uint32_t)(n - g) : 16u;
    // window of the step's first byte, and bytes left in it
    uint64_t w = (first + g) / window;
    uint64_t rem = window - (first + g) % window;
    for (uint32_t h = 0; h < lim; h++) {
      if (rem == 0) {
        w++;
        rem = window;
      }
      if (w != cur_w) {
        if (acc && cur_w < n_counts) atomicAdd(&counts[cur_w], acc);
        cur_w = w;
        acc = 0;
      }
      acc += buf[g + h] == value ? 1ull : 0ull;
      rem--;
    }
  }
  if (acc && cur_w < n_counts) atomicAdd(&counts[cur_w], acc);
}

// ---------------------------------------------------------------------------
// Host-callable launchers
// ---------------------------------------------------------------------------

}  // namespace gzgpu

using namespace gzgpu;

// ---------------------------------------------------------------------------
// Workspace for the entry point that allocates nothing (gz_decompress_static):
// a static device array, one per GPU the library runs on, held until the
// process ends.  Host code must not use the array's name as an address: the
// device address of each GPU's copy is looked up once per device, with that
// device current, and cached.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

extern "C" {

// The current device's scratch address (looked up on the first call there).
hipError_t gzk_scratch(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = q;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t gzk_init(ChunkState *cs, uint32_t n_chunks, FileState *fs, uint32_t n_files, Counters *ctr,
                    hipStream_t st) {
  uint32_t n = n_chunks > n_files ? n_chunks : n_files;
  if (n < 16) n = 16;
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, st, cs, n_chunks, fs, n_files, ctr);
  return hipGetLastError();
}

hipError_t gzk_capacity(uint32_t n_files, const FileDesc *files, ChunkDesc *chunks, const ChunkState *cs,
                        uint32_t factor, hipStream_t st) {
  hipLaunchKernelGGL(k_capacity, dim3(n_files), dim3(CAP_THREADS), 0, st, files, chunks, cs, factor);
  return hipGetLastError();
}

hipError_t gzk_scan(const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs, const uint32_t *scan_list,
                    uint32_t n_scan, uint32_t groups, hipStream_t st) {
  if (n_scan == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(n_scan * groups), dim3(256), 0, st, files, chunks, cs, scan_list, n_scan, groups);
  return hipGetLastError();
}

#define GZ_WIN_SWITCH(win, CALL)   \
  switch (win) {                   \
    case 512: {                    \
      constexpr int W = 512;       \
      CALL;                        \
    } break;                       \
    case 1024: {                   \
      constexpr int W = 1024;      \
      CALL;                        \
    } break;                       \
    case 2048: {                   \
      constexpr int W = 2048;      \
      CALL;                        \
    } break;                       \
    case 4096: {                   \
      constexpr int W = 4096;      \
      CALL;                        \
    } break;                       \
    case 8192: {                   \
      constexpr int W = 8192;      \
      CALL;                        \
    } break;                       \
    case 16384: {                  \
      constexpr int W = 16384;     \
      CALL;                        \
    } break;                       \
    case 32768: {                  \
      constexpr int W = 32768;     \
      CALL;                        \
    } break;                       \
    default:                       \
      return hipErrorInvalidValue; \
  }

hipError_t gzk_inflate(int win, uint32_t stored, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks,
                       ChunkState *cs, const uint32_t *order, uint32_t n, Counters *ctr, uint16_t *pool, hipStream_t st) {
  if (stored) {
    GZ_WIN_SWITCH(win, hipLaunchKernelGGL((k_inflate<W, true>), dim3(grid), dim3(64), 0, st, files, chunks, cs, order,
                                          n, ctr, pool));
  } else {
    GZ_WIN_SWITCH(win, hipLaunchKernelGGL((k_inflate<W, false>), dim3(grid), dim3(64), 0, st, files, chunks, cs, order,
                                          n, ctr, pool));
  }
  return hipGetLastError();
}

hipError_t gzk_confirm(int win, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                       uint32_t n, Counters *ctr, uint16_t *pool, uint32_t always_decode, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_confirm<W>, dim3(grid), dim3(64), 0, st, files, chunks, cs, n, ctr, pool,
                                        always_decode));
  return hipGetLastError();
}

hipError_t gzk_redo(int win, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs, uint32_t n,
                    Counters *ctr, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_redo<W>, dim3(grid), dim3(64), 0, st, files, chunks, cs, n, ctr, pool));
  return hipGetLastError();
}

hipError_t gzk_stitch(int win, uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                      uint32_t n, Counters *ctr, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_stitch<W>, dim3(grid), dim3(64), 0, st, files, chunks, cs, n, ctr, pool));
  return hipGetLastError();
}

hipError_t gzk_finalize(int win, uint32_t n_files, const FileDesc *files, const ChunkDesc *chunks, ChunkState *cs,
                        FileState *fs, uint16_t *pool, hipStream_t st) {
  GZ_WIN_SWITCH(win, hipLaunchKernelGGL(k_finalize<W>, dim3(n_files), dim3(FIN_THREADS), 0, st, files, chunks, cs, fs, pool));
  return hipGetLastError();
}

hipError_t gzk_crc(uint32_t n_files, const FileDesc *files, FileState *fs, const uint32_t *xpow, uint64_t total_units,
                   hipStream_t st) {
  if (total_units) {
    hipLaunchKernelGGL(k_crc, dim3((uint32_t)((total_units + 3) / 4)), dim3(256), 0, st, files, n_files, fs, xpow,
                       total_units);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_crc_final, dim3(1), dim3(256), 0, st, files, n_files, fs, xpow);
  return hipGetLastError();
}

hipError_t gzk_tilescan(const ChunkDesc *chunks, const ChunkState *cs, const FileState *fs, uint32_t n, uint64_t *tiles,
                        uint32_t *acc_pos, AccEntry *acc, hipStream_t st) {
  hipLaunchKernelGGL(k_tilescan, dim3(1), dim3(1024), 0, st, chunks, cs, fs, n, tiles, acc_pos, acc);
  return hipGetLastError();
}

hipError_t gzk_propagate(uint32_t n, const uint32_t *acc_pos, const AccEntry *acc, uint8_t *wins, const uint16_t *pool,
                         uint16_t *maps, uint8_t *segwin, hipStream_t st) {
  const uint32_t smax = (n + PSEG - 1) / PSEG;
  hipLaunchKernelGGL(k_prop_maps, dim3(smax), dim3(PROP_THREADS), 0, st, acc_pos, n, acc, pool, wins, maps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // prefix compositions, alternating between the two map arrays
  uint16_t *cur = maps, *alt = maps + (uint64_t)smax * WINDOW;
  for (uint32_t dist = 1; dist + 1 < smax; dist *= 2) {
    hipLaunchKernelGGL(k_prop_scan, dim3(PROP_PARTS * smax), dim3(256), 0, st, acc_pos, n, cur, alt, dist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint16_t *t = cur;
    cur = alt;
    alt = t;
  }
  hipLaunchKernelGGL(k_prop_segwin, dim3(PROP_PARTS * smax), dim3(256), 0, st, acc_pos, n, acc, cur, wins, segwin);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prop_apply, dim3(smax), dim3(PROP_THREADS), 0, st, acc_pos, n, acc, pool, segwin, wins);
  return hipGetLastError();
}

hipError_t gzk_count_byte(const uint8_t *buf, uint64_t n, uint32_t value, uint64_t first, uint64_t window,
                         unsigned long long *counts, uint64_t n_counts, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t per = 16ull * 256;
  uint64_t blocks = (n + per - 1) / per;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_count_byte, dim3((uint32_t)blocks), dim3(256), 0, st, buf, n, value, first, window, counts,
                     n_counts);
  return hipGetLastError();
}

hipError_t gzk_carry(const FileDesc *files, const FileState *fs, const uint8_t *wins, uint8_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_carry, dim3(1), dim3(1024), 0, st, files, fs, wins, dst);
  return hipGetLastError();
}

hipError_t gzk_translate(uint32_t grid, const FileDesc *files, const ChunkDesc *chunks, const ChunkState *cs,
                         FileState *fs, const uint64_t *tiles, uint32_t n, const uint8_t *wins, const uint16_t *pool,
                         Counters *ctr, hipStream_t st) {
  hipLaunchKernelGGL(k_translate, dim3(grid), dim3(TRANSLATE_THREADS), 0, st, files, chunks, cs, fs, tiles, n, wins, pool, ctr);
  return hipGetLastError();
}

}  // extern "C"
