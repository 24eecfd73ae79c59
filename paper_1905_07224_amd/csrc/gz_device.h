// Device building blocks for the two-pass gzip path on gfx950 (CDNA4).
//
// A DEFLATE decoder that one 64-lane wavefront runs as a single sequential
// decoder: the bit position, the current symbol and all control flow are
// wave-uniform (scalar registers), the 64 lanes hold a 256-byte window of the
// compressed stream, build the Huffman lookup tables in LDS, copy matches and
// move output to HBM in coalesced 16-byte stores.
//
// Format: RFC 1951 (the paper defers to it in Section III).  Symbolic output:
// decompress(C_i, w_hat_i) of Section VI-C, where the context before a chunk
// is the 32768 unique symbols U_j, written 0x8000 | j.
#pragma once
#include <hip/hip_runtime.h>

#include "gz_internal.h"

namespace gzgpu {

// ---------------------------------------------------------------------------
// Small wave helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
// Orders LDS stores of some lanes before LDS loads of other lanes of the same
// wave.  A wave executes its LDS instructions in order, so this is only a
// compiler-level barrier on the GPU.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T uni(T v) {  // value of lane 0, as a scalar
  return (T)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool ascii_text(uint32_t c) {
  // printable ASCII of the block-start checks: TAB, LF, CR, 0x20..0x7E
  return c == 9u || c == 10u || c == 13u || (c >= 32u && c <= 126u);
}

// ---------------------------------------------------------------------------
// Compressed input.  Bit positions are counted from the first byte of the
// file.  The buffer may sit at any byte address: loads use the aligned dword
// that holds the byte and zero the bytes outside [0, n).  An aligned dword
// that contains at least one byte of the buffer lies in the same page as that
// byte, so these loads never leave mapped memory.
// ---------------------------------------------------------------------------

// Pointers to the input in the global address space, so that its loads are
// tracked apart from LDS traffic.
#ifndef GZ_GLOBAL
#define GZ_GLOBAL __attribute__((address_space(1)))
#endif
typedef const GZ_GLOBAL uint32_t *gdw_ptr;

// v_writelane_b32: `old` with lane l (uniform, below 64) replaced by the
// uniform value v.  hipcc has no builtin name for LLVM's amdgcn writelane
// intrinsic, so it is declared under the intrinsic's own name.
#ifndef GZ_WRITELANE
__device__ int gz_writelane_i32(int v, int l, int old) __asm("llvm.amdgcn.writelane.i32");
#define GZ_WRITELANE(v, l, old) gz_writelane_i32((v), (l), (old))
#endif

struct Src {
  gdw_ptr base;          // comp rounded down to 4 bytes
  uint32_t mis;          // comp & 3
  uint64_t nbytes;
  uint64_t end_bits;     // 8 * nbytes
  int64_t full_lo;       // dwords [full_lo, full_hi) lie wholly inside the buffer
  int64_t full_hi;

  __device__ void init(const uint8_t *comp, uint64_t n) {
    uintptr_t p = (uintptr_t)comp;
    mis = (uint32_t)(p & 3u);
    base = (gdw_ptr)(p - mis);
    nbytes = n;
    end_bits = 8ull * n;
    full_lo = mis ? 1 : 0;
    full_hi = (int64_t)((mis + n) >> 2);
  }
  // a dword at an edge of the buffer: bytes outside [0, n) read as zero
  __device__ uint32_t dw_edge(int64_t D) const {
    int64_t b0 = D * 4 - (int64_t)mis;
    if (b0 + 4 <= 0 || b0 >= (int64_t)nbytes) return 0u;
    uint32_t w = base[D];
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (b0 + k >= 0 && b0 + k < (int64_t)nbytes) m |= 0xFFu << (8 * k);
    return w & m;
  }
  // dword D of the aligned view (file bytes 4D - mis .. 4D - mis + 3)
  __device__ __forceinline__ uint32_t dw(int64_t D) const {
    if (D >= full_lo && D < full_hi) return base[D];
    return dw_edge(D);
  }
  // 64 bits starting at file bit b (bits past the end read as zero); per lane
  __device__ __forceinline__ uint64_t peek64(uint64_t b) const {
    uint64_t a = b + 8ull * mis;
    int64_t D = (int64_t)(a >> 5);
    uint32_t s = (uint32_t)(a & 31);
    uint64_t lo = ((uint64_t)dw(D + 1) << 32) | dw(D);
    uint64_t hi = dw(D + 2);
    return s ? ((lo >> s) | (hi << (64 - s))) : lo;
  }
  __device__ __forceinline__ uint32_t byte(uint64_t fb) const {
    uint64_t a = fb + mis;
    return (dw((int64_t)(a >> 2)) >> (8 * (a & 3))) & 0xFFu;
  }
};

// ---------------------------------------------------------------------------
// Wave-uniform bit reader.  Lane l holds the dword D of the aligned view with
// D = l (mod 64) for D in [lo, lo + 64); lo is a multiple of 32.  refill(),
// called before each peek(), moves the window when the read position has
// entered the upper half: the lanes of the consumed half take the dwords
// prefetched one half earlier and prefetch the next ones, so a refill never
// waits on memory.  A symbol with its extra bits takes at most 48 bits, so one
// peek() after a refill always has 64 valid bits.
// ---------------------------------------------------------------------------

struct WaveBits {
  Src s;
  uint64_t pos;  // file bit position (uniform)
  int64_t lo;    // first dword held (uniform)
  uint32_t win;  // per lane
  uint32_t nxt;  // per lane

  __device__ __forceinline__ int64_t dword_of(uint64_t p) const { return (int64_t)((p + 8ull * s.mis) >> 5); }

  __device__ void init(uint64_t p) {
    pos = p;
    lo = dword_of(p) & ~31ll;
    int l = lane_id();
    int64_t D = lo + ((l - (int)(lo & 63)) & 63);
    win = s.dw(D);
    nxt = (D < lo + 32) ? s.dw(D + 64) : 0u;
  }
  __device__ void half_step() {
    int l = lane_id();
    int64_t Dl = lo + ((l - (int)(lo & 63)) & 63);
    win = Dl < lo + 32 ? nxt : win;
    lo += 32;
    int64_t D2 = lo + ((l - (int)(lo & 63)) & 63);
    if (D2 < lo + 32) nxt = s.dw(D2 + 64);
  }
  __device__ __forceinline__ void refill() {
    const int64_t D = dword_of(pos);
    if (D >= lo + 32) {
      if (D >= lo + 48) init(pos);  // a jump (stored block)
      else half_step();
    }
  }
  // 64 bits at pos; valid after refill() and until 48 more bits are skipped
  __device__ __forceinline__ uint64_t peek() const {
    uint64_t a = pos + 8ull * s.mis;
    int64_t D = (int64_t)(a >> 5);
    uint32_t sh = (uint32_t)(a & 31);
    uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)win, (int)(D & 63));
    uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)win, (int)((D + 1) & 63));
    uint32_t w2 = (uint32_t)__builtin_amdgcn_readlane((int)win, (int)((D + 2) & 63));
    uint64_t v = ((uint64_t)w1 << 32) | w0;
    return sh ? ((v >> sh) | ((uint64_t)w2 << (64 - sh))) : v;
  }
  __device__ __forceinline__ uint64_t next() {
    refill();
    return peek();
  }
  // 192 bits at pos as six dwords (q[0] holds bits pos .. pos + 31)
  __device__ __forceinline__ void view192(uint32_t (&q)[6]) {
    refill();
    const uint64_t a = pos + 8ull * s.mis;
    const int64_t D = (int64_t)(a >> 5);
    const uint32_t sh = (uint32_t)(a & 31);
    uint32_t w[7];
#pragma unroll
    for (int i = 0; i < 7; i++) w[i] = (uint32_t)__builtin_amdgcn_readlane((int)win, (int)((D + i) & 63));
#pragma unroll
    for (int i = 0; i < 6; i++) q[i] = (uint32_t)((((uint64_t)w[i + 1] << 32) | w[i]) >> sh);
  }
  // Per lane k: the 64 stream bits from pos + k (wa) and from pos + 64 + k
  // (wb), gathered with one ds_bpermute per dword from the lanes that hold
  // them (dwords D .. D + 6 of pos lie in the window after refill(), and
  // lanes are indexed by dword mod 64, so the low 32 bits of the position
  // suffice).  All vector work: no value goes through scalar registers.
  __device__ __forceinline__ void lane_windows(uint64_t &wa, uint64_t &wb) {
    refill();
    const uint32_t ak = (uint32_t)pos + 8u * s.mis + (uint32_t)lane_id();
    const uint32_t sh = ak & 31u;
    const uint32_t d = ak >> 5;
    uint32_t x[5];
#pragma unroll
    for (int i = 0; i < 5; i++) x[i] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(((d + (uint32_t)i) & 63u) << 2), (int)win);
    wa = ((uint64_t)__builtin_amdgcn_alignbit(x[2], x[1], sh) << 32) | __builtin_amdgcn_alignbit(x[1], x[0], sh);
    wb = ((uint64_t)__builtin_amdgcn_alignbit(x[4], x[3], sh) << 32) | __builtin_amdgcn_alignbit(x[3], x[2], sh);
  }
  __device__ __forceinline__ void skip(uint32_t n) { pos += n; }
  __device__ __forceinline__ bool past_end() const { return pos > s.end_bits; }
};

// ---------------------------------------------------------------------------
// Huffman lookup tables (RFC 1951 section 3.2.2 canonical codes).
//
// Distance (and code-length) entries: [3:0] code length, [7:4] kind, [15:8]
// extra bits (code-length codes: the symbol), [31:16] base distance.
//
// Literal/length entries are the decoder's token words wherever the code
// alone fixes the token: [7:0] bits used, [16:8] output symbols, [31:17]
// payload.  A literal: 1 output symbol, the byte in [24:17], and bit 31 set
// when the byte is outside the block-start check's ASCII set.  A special
// token has 448 output symbols and its kind in [31:17] (end-of-block: its
// code length in [7:0]).  A length code, whose token also depends on the
// bits that follow it, has 0 output symbols: [3:0] code length, [7:4] extra
// bits, [25:17] base length.
// ---------------------------------------------------------------------------

enum : uint32_t { K_LEN = 1, K_LONG = 3, K_BAD = 4, K_BADSYM = 5 };

constexpr uint32_t TOK_SPECIAL = 448u << 8;
constexpr uint32_t TOK_EOB = TOK_SPECIAL | (1u << 17);
constexpr uint32_t TOK_SLOW = TOK_SPECIAL | (2u << 17);    // a code longer than the table: decoded alone
constexpr uint32_t TOK_ASCII = TOK_SPECIAL | (3u << 17);   // (decoder only) a non-ASCII literal in a checked block
constexpr uint32_t TOK_BADSYM = TOK_SPECIAL | (4u << 17);  // literal/length 286, 287, or no code at all
constexpr uint32_t TOK_NONASCII = 1u << 31;

constexpr int LIT_BITS = 10;
constexpr int DIST_BITS = 9;
constexpr int CL_BITS = 7;

// lengths 3..258 (section 3.2.5): codes 257..264 carry no extra bits, then
// four codes per extra-bit count 1..5, then 285 = 258
__device__ __forceinline__ uint32_t litlen_entry(uint32_t sym, uint32_t len) {
  if (sym < 256u) return len | (1u << 8) | (sym << 17) | (ascii_text(sym) ? 0u : TOK_NONASCII);
  if (sym == 256u) return TOK_EOB | len;
  if (sym <= 285u) {
    uint32_t i = sym - 257u, ex, base;
    if (i < 8u) {
      ex = 0;
      base = 3u + i;
    } else if (i == 28u) {
      ex = 0;
      base = 258u;
    } else {
      ex = (i - 4u) >> 2;
      base = ((4u + (i & 3u)) << ex) + 3u;
    }
    return len | (ex << 4) | (base << 17);
  }
  return TOK_BADSYM;
}
// distances 1..32768: codes 0..3 exact, then two codes per extra-bit count 1..13
__device__ __forceinline__ uint32_t dist_entry(uint32_t sym, uint32_t len) {
  if (sym < 30u) {
    uint32_t ex, base;
    if (sym < 4u) {
      ex = 0;
      base = sym + 1u;
    } else {
      ex = (sym >> 1) - 1u;
      base = ((2u + (sym & 1u)) << ex) + 1u;
    }
    return len | (K_LEN << 4) | (ex << 8) | (base << 16);
  }
  return len | (K_BADSYM << 4);
}
__device__ __forceinline__ uint32_t cl_entry(uint32_t sym, uint32_t len) { return len | (sym << 8); }

struct TreeInfo {
  uint16_t first[16];  // first canonical code of each length
  uint16_t count[16];
  uint16_t base[16];   // index of the first symbol of each length in the sorted list
};

enum TreeKind { TREE_LIT = 0, TREE_DIST = 1, TREE_CL = 2 };

// Per-tree build, run by the whole wave.  lens: n code lengths in LDS.
// Returns the Kraft remainder scaled by 2^15 (0 complete, > 0 incomplete,
// < 0 over-subscribed) and the number of codes.  With fill, also writes the
// sorted symbol list, the per-length info and the 2^LB-entry lookup table
// (codes longer than LB get K_LONG, unused bit patterns K_BAD; in the
// literal/length table TOK_SLOW and TOK_BADSYM).
template <int LB, int KIND>
__device__ int build_tree(const uint8_t *lens, int n, uint32_t *tab, TreeInfo *ti, uint16_t *sorted, int *ncodes,
                          bool fill) {
  const int lane = lane_id();
  int cnt[16];
#pragma unroll
  for (int l = 0; l < 16; l++) cnt[l] = 0;
  for (int b = 0; b < n; b += 64) {
    int s = b + lane;
    int L = s < n ? (int)lens[s] : 0;
#pragma unroll
    for (int l = 1; l < 16; l++) cnt[l] += __popcll(__ballot(L == l));
  }
  int nc = 0, left = 32768;
#pragma unroll
  for (int l = 1; l < 16; l++) {
    nc += cnt[l];
    left -= cnt[l] << (15 - l);
  }
  *ncodes = nc;
  if (!fill || left < 0) return left;
  int first[16], base[16];
  {
    int code = 0, b = 0;
    first[0] = 0;
    base[0] = 0;
#pragma unroll
    for (int l = 1; l < 16; l++) {
      code = (code + (l > 1 ? cnt[l - 1] : 0)) << 1;
      first[l] = code;
      base[l] = b;
      b += cnt[l];
    }
  }
  if (lane < 16) {
    int f = 0, c = 0, bb = 0;
#pragma unroll
    for (int l = 0; l < 16; l++)
      if (lane == l) {
        f = first[l];
        c = cnt[l];
        bb = base[l];
      }
    ti->first[lane] = (uint16_t)f;
    ti->count[lane] = (uint16_t)c;
    ti->base[lane] = (uint16_t)bb;
  }
  // symbols in (length, value) order
  {
    int run[16];
#pragma unroll
    for (int l = 0; l < 16; l++) run[l] = base[l];
    const uint64_t below = lanes_below();
    for (int b = 0; b < n; b += 64) {
      int s = b + lane;
      int L = s < n ? (int)lens[s] : 0;
      int at = -1;
#pragma unroll
      for (int l = 1; l < 16; l++) {
        uint64_t m = __ballot(L == l);
        if (L == l) at = run[l] + __popcll(m & below);
        run[l] += __popcll(m);
      }
      if (at >= 0) sorted[at] = (uint16_t)s;
    }
  }
  wave_sync();
  // lookup table: the LB-bit prefix P (first bit read = most significant)
  // falls in the left-justified code interval of exactly one length
  const int endLB = (first[LB] + cnt[LB]);  // in LB-bit units
  const int end15 = first[15] + cnt[15];    // in 15-bit units
  for (int x = lane; x < (1 << LB); x += 64) {
    int P = (int)(__builtin_bitreverse32((uint32_t)x) >> (32 - LB));
    uint32_t e;
    if (P < endLB) {
      int idx = 0, len = 0;
      bool done = false;
#pragma unroll
      for (int l = 1; l <= LB; l++) {
        int endl = (first[l] + cnt[l]) << (LB - l);
        if (!done && P < endl) {
          idx = base[l] + (P >> (LB - l)) - first[l];
          len = l;
          done = true;
        }
      }
      uint32_t sym = sorted[idx];
      e = KIND == TREE_LIT ? litlen_entry(sym, (uint32_t)len)
          : KIND == TREE_DIST ? dist_entry(sym, (uint32_t)len)
                              : cl_entry(sym, (uint32_t)len);
    } else if ((P << (15 - LB)) < end15) {
      e = KIND == TREE_LIT ? TOK_SLOW : K_LONG << 4;
    } else {
      e = KIND == TREE_LIT ? TOK_BADSYM : K_BAD << 4;
    }
    tab[x] = e;
  }
  wave_sync();
  return left;
}

// Codes longer than the table: compare the 15-bit prefix against each length.
template <int LB, int KIND>
__device__ __forceinline__ uint32_t decode_long(uint64_t v, const TreeInfo *ti, const uint16_t *sorted) {
  uint32_t r = __builtin_bitreverse32((uint32_t)v) >> 17;  // next 15 bits, first bit most significant
  for (int l = LB + 1; l <= 15; l++) {
    uint32_t c = r >> (15 - l);
    uint32_t f = uni32(ti->first[l]), n = uni32(ti->count[l]);
    if (c - f < n) {
      uint32_t sym = uni32(sorted[uni32(ti->base[l]) + (c - f)]);
      return KIND == TREE_LIT ? litlen_entry(sym, (uint32_t)l) : dist_entry(sym, (uint32_t)l);
    }
  }
  return KIND == TREE_LIT ? TOK_BADSYM : K_BAD << 4;
}

// ---------------------------------------------------------------------------
// Per-wave LDS
// ---------------------------------------------------------------------------

struct TablesLDS {
  uint32_t lit[1 << LIT_BITS];
  uint32_t dist[1 << DIST_BITS];  // also holds the code-length code table while lengths are read
  uint16_t lsorted[288];
  uint16_t dsorted[32];
  TreeInfo li;
  TreeInfo di;
  uint8_t lens[320];
};

// reasons (only their class matters: a candidate is rejected, or data is invalid)
enum : int { D_OK = 0, D_BAD = 1, D_TRUNC = 2, D_ASCII = 3, D_SIZE = 4, D_FAR = 5, D_STATIC = 6 };

// Dynamic-block code tables (section 3.2.7).  strict: the literal/length code
// must be complete (block-start checks); otherwise one lone 1-bit code is also
// accepted.  fill = false only validates.
__device__ int read_dynamic_tables(WaveBits &br, TablesLDS &sh, bool strict, bool fill, bool *no_dist) {
  const int lane = lane_id();
  uint64_t v = br.next();
  const uint32_t hlit = (uint32_t)(v & 31u) + 257u;
  const uint32_t hdist = (uint32_t)((v >> 5) & 31u) + 1u;
  const uint32_t hclen = (uint32_t)((v >> 10) & 15u) + 4u;
  br.skip(14);
  if (hlit > 286u || hdist > 30u) return D_BAD;
  v = br.next();
  // code-length code lengths, sent in the order 16 17 18 0 8 7 9 6 10 5 11 4 12 3 13 2 14 1 15
  if (lane < 19) sh.lens[lane] = 0;
  wave_sync();
  if (lane < (int)hclen) {
    // position of lane's entry in that order, as 5-bit fields
    const uint64_t ord_lo = (16ull) | (17ull << 5) | (18ull << 10) | (0ull << 15) | (8ull << 20) | (7ull << 25) |
                            (9ull << 30) | (6ull << 35) | (10ull << 40) | (5ull << 45) | (11ull << 50) |
                            (4ull << 55);
    const uint64_t ord_hi = (12ull) | (3ull << 5) | (13ull << 10) | (2ull << 15) | (14ull << 20) | (1ull << 25) |
                            (15ull << 30);
    uint32_t sym = lane < 12 ? (uint32_t)((ord_lo >> (5 * lane)) & 31u) : (uint32_t)((ord_hi >> (5 * (lane - 12))) & 31u);
    sh.lens[sym] = (uint8_t)((v >> (3 * lane)) & 7u);
  }
  br.skip(3 * hclen);
  wave_sync();
  int ncl;
  int left = build_tree<CL_BITS, TREE_CL>(sh.lens, 19, sh.dist, &sh.di, sh.dsorted, &ncl, true);
  if (left != 0) return D_BAD;  // code-length code over-subscribed or incomplete
  const uint32_t total = hlit + hdist;
  uint32_t i = 0, prev = 0;
  int lit_left = 32768, dist_left = 32768;
  // every pass stores at least one length, so total passes at most
  for (uint32_t pass = 0; i < total; pass++) {
    if (pass >= total) return D_BAD;
    v = br.next();
    const uint32_t e = uni32(sh.dist[v & 127u]);
    uint32_t cl = e & 15u, sym = e >> 8;
    if (sym < 16u) {
      if (lane == 0) sh.lens[i] = (uint8_t)sym;
      if (sym) {
        if (i < hlit) lit_left -= 1 << (15 - sym);
        else dist_left -= 1 << (15 - sym);
      }
      prev = sym;
      i++;
      br.skip(cl);
    } else {
      uint32_t rep, val;
      if (sym == 16u) {
        if (i == 0) return D_BAD;
        rep = 3u + (uint32_t)((v >> cl) & 3u);
        val = prev;
        br.skip(cl + 2);
      } else if (sym == 17u) {
        rep = 3u + (uint32_t)((v >> cl) & 7u);
        val = 0;
        br.skip(cl + 3);
      } else {
        rep = 11u + (uint32_t)((v >> cl) & 127u);
        val = 0;
        br.skip(cl + 7);
      }
      if (i + rep > total) return D_BAD;
      for (uint32_t k = (uint32_t)lane; k < rep; k += 64) sh.lens[i + k] = (uint8_t)val;
      if (val) {
        uint32_t nl = i < hlit ? min(i + rep, hlit) - i : 0u;
        lit_left -= (int)nl << (15 - val);
        dist_left -= (int)(rep - nl) << (15 - val);
      }
      prev = val;
      i += rep;
    }
    if (br.past_end()) return D_TRUNC;
    if (lit_left < 0 || dist_left < 0) return D_BAD;
  }
  wave_sync();
  if (uni32(sh.lens[256]) == 0) return D_BAD;  // no end-of-block code
  int nlit, ndist;
  left = build_tree<LIT_BITS, TREE_LIT>(sh.lens, (int)hlit, sh.lit, &sh.li, sh.lsorted, &nlit, fill);
  if (left < 0) return D_BAD;
  if (left > 0) {
    bool lone = nlit == 1 && uni32(sh.lens[256]) == 1;  // only end-of-block, one bit
    if (strict || !lone) return D_BAD;
  }
  left = build_tree<DIST_BITS, TREE_DIST>(sh.lens + hlit, (int)hdist, sh.dist, &sh.di, sh.dsorted, &ndist, fill);
  if (left < 0) return D_BAD;
  *no_dist = ndist == 0;
  if (left > 0 && ndist != 0) {
    bool lone = false;
    if (ndist == 1) {
      // the one code must be 1 bit long
      int one = 0;
      for (uint32_t k = (uint32_t)lane; k < hdist; k += 64) one |= sh.lens[hlit + k] == 1;
      lone = __ballot(one) != 0;
    }
    if (!lone) return D_BAD;
  }
  return D_OK;
}

__device__ __forceinline__ void fixed_tables(TablesLDS &sh) {
  const int lane = lane_id();
  for (int s = lane; s < 288; s += 64) sh.lens[s] = (uint8_t)(s < 144 ? 8 : s < 256 ? 9 : s < 280 ? 7 : 8);
  wave_sync();
  int n;
  build_tree<LIT_BITS, TREE_LIT>(sh.lens, 288, sh.lit, &sh.li, sh.lsorted, &n, true);
  if (lane < 32) sh.lens[lane] = 5;
  wave_sync();
  build_tree<DIST_BITS, TREE_DIST>(sh.lens, 32, sh.dist, &sh.di, sh.dsorted, &n, true);
}

// ---------------------------------------------------------------------------
// Block-start checks of Appendix A, cheap stage: one lane per candidate bit.
// BFINAL = 0, BTYPE = 10, HLIT <= 286, HDIST <= 30, complete code-length code.
// With FD_STORED_STARTS also a stored block: BFINAL = 0, BTYPE = 00, zero
// padding to the byte boundary, LEN and NLEN complements, LEN > 1024 (the
// trial block's size bound); that is its whole static check.
// ---------------------------------------------------------------------------

// v: the 64 stream bits from b (b's bit first)
__device__ __forceinline__ bool stored_start_bits(uint64_t v, uint64_t b, uint64_t end_bits) {
  const uint32_t pad = (uint32_t)(((b + 10u) & ~7ull) - b);  // header and padding bits, 3..10
  if (b + pad + 32u > end_bits) return false;
  if (v & ((1ull << pad) - 1ull)) return false;
  const uint32_t x = (uint32_t)(v >> pad);
  const uint32_t len = x & 0xFFFFu;
  return (len ^ 0xFFFFu) == (x >> 16) && len > 1024u;
}

__device__ __forceinline__ bool stored_start_at(const Src &s, uint64_t b) {
  return stored_start_bits(s.peek64(b), b, s.end_bits);
}

template <bool STORED>
__device__ __forceinline__ bool start_stage1(const Src &s, uint64_t b, uint32_t mode) {
  if (b + 17 > s.end_bits) return STORED && (mode & FD_STORED_STARTS) && b < s.end_bits && stored_start_at(s, b);
  uint64_t v = s.peek64(b);
  if (STORED && (mode & FD_STORED_STARTS) && (v & 7u) == 0u) return stored_start_at(s, b);
  if ((v & 7u) != 4u) return false;
  if (((v >> 3) & 31u) > 29u || ((v >> 8) & 31u) > 29u) return false;
  uint32_t hclen = (uint32_t)((v >> 13) & 15u) + 4u;
  uint64_t w = s.peek64(b + 17);
  int left = 128;
  for (uint32_t i = 0; i < hclen; i++) {
    uint32_t L = (uint32_t)(w >> (3 * i)) & 7u;
    if (L) left -= 128 >> L;
  }
  return left == 0;
}

// Kraft sums of three code-length code lengths at once: entry i (9 bits,
// three 3-bit lengths) is the sum of 128 >> L over its nonzero lengths L.
__device__ __forceinline__ void kraft3_fill(uint8_t *k3, int tid, int nthreads) {
  for (int i = tid; i < 512; i += nthreads) {
    uint32_t v = 0;
    for (int f = 0; f < 3; f++) {
      const uint32_t L = ((uint32_t)i >> (3 * f)) & 7u;
      if (L) v += 128u >> L;
    }
    k3[i] = (uint8_t)v;
  }
}

// The cheap stage for the 32 candidates of one aligned dword (dword W of the
// aligned view; its bit k is file bit 32 * W + k - 8 * mis), in three parts.
// x0..x3: dwords W .. W + 3 (zero past the buffer).
//
// stage1_header_mask: the positions where BFINAL = 0, BTYPE = 10, HLIT <= 29
// and HDIST <= 29, all 32 tested with word operations (a 5-bit count is 30
// or 31 exactly when its upper four bits are set).
__device__ __forceinline__ uint32_t stage1_header_mask(uint32_t x0, uint32_t x1) {
  const uint64_t lo = ((uint64_t)x1 << 32) | x0;
  const uint64_t hlit_hi = (lo >> 4) & (lo >> 5) & (lo >> 6) & (lo >> 7);
  const uint64_t hdist_hi = (lo >> 9) & (lo >> 10) & (lo >> 11) & (lo >> 12);
  return (uint32_t)(~lo & ~(lo >> 1) & (lo >> 2) & ~hlit_hi & ~hdist_hi);
}

// stage1_kraft_ok: for one position k with a passing header, whether the
// code-length code is complete; its Kraft sum takes seven lookups in k3
// (kraft3_fill) over the 3-bit lengths from bit 17 on, HCLEN of them.
__device__ __forceinline__ bool stage1_kraft_ok(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t k,
                                                const uint8_t *k3) {
  const uint32_t w0 = __builtin_amdgcn_alignbit(x1, x0, k);
  const uint32_t w1 = __builtin_amdgcn_alignbit(x2, x1, k);
  const uint32_t w2 = __builtin_amdgcn_alignbit(x3, x2, k);
  const uint32_t hclen = ((w0 >> 13) & 15u) + 4u;
  const uint64_t cl = ((uint64_t)(w0 >> 17) | ((uint64_t)w1 << 15) | ((uint64_t)w2 << 47)) &
                      ((1ull << (3 * hclen)) - 1ull);
  const uint32_t sum = (uint32_t)k3[cl & 511u] + k3[(cl >> 9) & 511u] + k3[(cl >> 18) & 511u] +
                       k3[(cl >> 27) & 511u] + k3[(cl >> 36) & 511u] + k3[(cl >> 45) & 511u] + k3[cl >> 54];
  return sum == 128u;
}

// stage1_stored_mask (FD_STORED_STARTS only): the positions where BFINAL = 0,
// BTYPE = 00 and the padding and LEN/NLEN pass (they lie within the four
// dwords: a byte boundary of the view is one of the file).
__device__ __forceinline__ uint32_t stage1_stored_mask(const Src &s, int64_t W, uint32_t x0, uint32_t x1, uint32_t x2,
                                                       uint32_t x3) {
  const uint64_t lo = ((uint64_t)x1 << 32) | x0;
  const uint64_t hi = ((uint64_t)x3 << 32) | x2;
  uint32_t sp = (uint32_t)(~lo & ~(lo >> 1) & ~(lo >> 2));
  uint32_t pass = 0;
  for (int g = 0; g < 32 && sp; g++) {
    const uint32_t k = (uint32_t)__builtin_ctz(sp);
    sp &= sp - 1;
    const int64_t b = 32 * W + (int64_t)k - 8 * (int64_t)s.mis;
    if (b < 0) continue;
    const uint64_t v = (lo >> k) | (k ? hi << (64 - k) : 0ull);
    if (stored_start_bits(v, (uint64_t)b, s.end_bits)) pass |= 1u << k;
  }
  return pass;
}

// Bits k of a dword whose file bit b0 + k lies in [lo, hi).
__device__ __forceinline__ uint32_t bits_in(int64_t b0, int64_t lo, int64_t hi) {
  const int64_t klo = std::min<int64_t>(32, std::max<int64_t>(0, lo - b0));
  const int64_t khi = std::min<int64_t>(32, std::max<int64_t>(0, hi - b0));
  return khi > klo ? (uint32_t)(((1ull << (khi - klo)) - 1ull) << klo) : 0u;
}

// The checks of read_dynamic_tables(strict, nothing stored), with the
// code-length symbols decoded speculatively: in a round of 128 bit offsets
// lane k decodes the symbol that would start at offset k and at k + 64 (one
// lookup each in the code-length table, extra bits included), then a scalar
// walk follows the real symbols from offset 0.  The walk keeps what the
// final checks need (the Kraft sums of the literal/length and distance
// codes, the end-of-block code's length, the number of distance codes and
// of 1-bit ones), so no code length is stored and no table is built.
__device__ __forceinline__ uint32_t cl_symbol_word(uint32_t bits, const TablesLDS &sh) {
  const uint32_t e = sh.dist[bits & 127u];
  const uint32_t cl = e & 15u, sym = e >> 8;
  const uint32_t ex = sym == 16u ? 2u : sym == 17u ? 3u : sym == 18u ? 7u : 0u;
  const uint32_t extra = (bits >> cl) & ((1u << ex) - 1u);
  return (cl + ex) | (sym << 4) | (extra << 9);  // bits used, symbol, extra value
}

__device__ int check_dynamic_tables(WaveBits &br, TablesLDS &sh) {
  const int lane = lane_id();
  uint64_t v = br.next();
  const uint32_t hlit = (uint32_t)(v & 31u) + 257u;
  const uint32_t hdist = (uint32_t)((v >> 5) & 31u) + 1u;
  const uint32_t hclen = (uint32_t)((v >> 10) & 15u) + 4u;
  br.skip(14);
  if (hlit > 286u || hdist > 30u) return D_BAD;
  v = br.next();
  if (lane < 19) sh.lens[lane] = 0;
  wave_sync();
  if (lane < (int)hclen) {
    const uint64_t ord_lo = (16ull) | (17ull << 5) | (18ull << 10) | (0ull << 15) | (8ull << 20) | (7ull << 25) |
                            (9ull << 30) | (6ull << 35) | (10ull << 40) | (5ull << 45) | (11ull << 50) |
                            (4ull << 55);
    const uint64_t ord_hi = (12ull) | (3ull << 5) | (13ull << 10) | (2ull << 15) | (14ull << 20) | (1ull << 25) |
                            (15ull << 30);
    uint32_t sym = lane < 12 ? (uint32_t)((ord_lo >> (5 * lane)) & 31u) : (uint32_t)((ord_hi >> (5 * (lane - 12))) & 31u);
    sh.lens[sym] = (uint8_t)((v >> (3 * lane)) & 7u);
  }
  br.skip(3 * hclen);
  wave_sync();
  int ncl;
  if (build_tree<CL_BITS, TREE_CL>(sh.lens, 19, sh.dist, &sh.di, sh.dsorted, &ncl, true) != 0) return D_BAD;
  wave_sync();
  const uint32_t total = hlit + hdist;
  uint32_t i = 0, prev = 0, eob = 0, ndist = 0, d1 = 0;
  int lit_left = 32768, dist_left = 32768;
  const uint32_t sh5 = (uint32_t)lane & 31u;
  const bool lo_half = lane < 32;
  while (i < total) {
    uint32_t q[6];
    br.view192(q);
    const uint32_t ta = cl_symbol_word(lo_half ? __builtin_amdgcn_alignbit(q[1], q[0], sh5)
                                               : __builtin_amdgcn_alignbit(q[2], q[1], sh5), sh);
    const uint32_t tb = cl_symbol_word(lo_half ? __builtin_amdgcn_alignbit(q[3], q[2], sh5)
                                               : __builtin_amdgcn_alignbit(q[4], q[3], sh5), sh);
    uint32_t off = 0;
    while (off < 128u && i < total) {
      const uint32_t t = (uint32_t)__builtin_amdgcn_readlane(off < 64u ? (int)ta : (int)tb, (int)(off & 63u));
      const uint32_t sym = (t >> 4) & 31u, extra = t >> 9;
      uint32_t L, n;
      if (sym < 16u) {
        L = sym;
        n = 1;
      } else if (sym == 16u) {
        if (i == 0) return D_BAD;
        L = prev;
        n = 3u + extra;
      } else {
        L = 0;
        n = (sym == 17u ? 3u : 11u) + extra;
      }
      if (i + n > total) return D_BAD;
      if (L) {
        const uint32_t nl = i < hlit ? min(i + n, hlit) - i : 0u;
        lit_left -= (int)nl << (15 - L);
        dist_left -= (int)(n - nl) << (15 - L);
        ndist += n - nl;
        if (L == 1u) d1 += n - nl;
      }
      if (i <= 256u && 256u < i + n) eob = L;
      prev = L;
      i += n;
      off += t & 15u;
      if (br.pos + off > br.s.end_bits) return D_TRUNC;
      if (lit_left < 0 || dist_left < 0) return D_BAD;
    }
    br.skip(off);
  }
  if (eob == 0) return D_BAD;                  // no end-of-block code
  if (lit_left != 0) return D_BAD;             // literal/length code incomplete
  if (dist_left > 0 && ndist != 0 && !(ndist == 1u && d1 == 1u)) return D_BAD;
  return D_OK;
}

// The same checks as check_dynamic_tables for one candidate per lane, with
// no wave operation (lanes check different candidates): the code-length
// code's lookup table is built by the lane in its own column of `tab`
// (128 entries, entry x at tab[64 * x + lane]: symbol | length << 5), and
// the code lengths are read through a per-lane 64-bit bit buffer, with the
// dword after it loaded one refill ahead (so a refill does not wait for
// memory).
struct LaneBits {
  const Src *s;
  int64_t D;     // aligned dword after nxt
  uint64_t acc;  // unread bits, first one in bit 0
  uint32_t nxt;  // the dword after acc's bits
  uint32_t n;    // bits in acc (>= 32 after every refill)
  uint64_t pos;  // file bit of acc's bit 0
  __device__ __forceinline__ void init(const Src &src, uint64_t b) {
    s = &src;
    const uint64_t a = b + 8ull * src.mis;
    D = (int64_t)(a >> 5);
    const uint32_t sh = (uint32_t)(a & 31);
    const uint32_t d0 = src.dw(D), d1 = src.dw(D + 1);
    nxt = src.dw(D + 2);
    D += 3;
    acc = ((uint64_t)d0 >> sh) | ((uint64_t)d1 << (32 - sh));
    n = 64 - sh;
    pos = b;
  }
  __device__ __forceinline__ void skip(uint32_t k) {
    acc >>= k;
    n -= k;
    pos += k;
    if (n < 32) {
      acc |= (uint64_t)nxt << n;
      n += 32;
      nxt = s->dw(D);
      D++;
    }
  }
};

__device__ __forceinline__ bool lane_tables_ok(const Src &s, uint64_t b, uint8_t *tab, int lane, uint32_t mode) {
  // a stored candidate passed its whole static check in stage 1
  if ((mode & FD_STORED_STARTS) && ((s.peek64(b) >> 1) & 3u) == 0u) return true;
  LaneBits br;
  br.init(s, b + 3);
  const uint32_t hlit = (uint32_t)(br.acc & 31u) + 257u;
  const uint32_t hdist = (uint32_t)((br.acc >> 5) & 31u) + 1u;
  const uint32_t hclen = (uint32_t)((br.acc >> 10) & 15u) + 4u;
  br.skip(14);
  if (hlit > 286u || hdist > 30u) return false;
  // code-length code lengths by symbol, 3 bits each (order 16 17 18 0 8 7 9
  // 6 10 5 11 4 12 3 13 2 14 1 15 in the stream)
  // (the buffer holds at least 32 bits: the lengths are read as up to 10,
  // then up to 9 more)
  const uint32_t h1 = hclen < 10u ? hclen : 10u, h2 = hclen - h1;
  uint64_t w = br.acc & ((1ull << (3 * h1)) - 1ull);
  br.skip(3 * h1);
  w |= (br.acc & ((1ull << (3 * h2)) - 1ull)) << 30;
  br.skip(3 * h2);
  const uint8_t order[19] = {16, 17, 18, 0, 8, 7, 9, 6, 10, 5, 11, 4, 12, 3, 13, 2, 14, 1, 15};
  uint64_t bysym = 0;
#pragma unroll
  for (int i = 0; i < 19; i++) bysym |= ((w >> (3 * i)) & 7ull) << (3 * order[i]);
  // lengths per length value (8 bits each), the Kraft sum, first codes
  uint64_t cnt = 0;
#pragma unroll
  for (int sy = 0; sy < 19; sy++) {
    const uint32_t L = (uint32_t)(bysym >> (3 * sy)) & 7u;
    cnt += L ? 1ull << (8 * L) : 0ull;
  }
  uint32_t kraft = 0;
  uint64_t next = 0;  // next code of each length (8 bits each)
  uint32_t code = 0;
#pragma unroll
  for (int L = 1; L <= 7; L++) {
    const uint32_t c = (uint32_t)(cnt >> (8 * L)) & 255u;
    kraft += c << (7 - L);
    code = (code + (L > 1 ? (uint32_t)(cnt >> (8 * (L - 1))) & 255u : 0u)) << 1;
    next |= (uint64_t)code << (8 * L);
  }
  if (kraft != 128u) return false;
  // the lane's table: every 7-bit index whose first L stream bits are the
  // symbol's code (read first bit first) holds the symbol
  for (int sy = 0; sy < 19; sy++) {
    const uint32_t L = (uint32_t)(bysym >> (3 * sy)) & 7u;
    if (!L) continue;
    const uint32_t c = (uint32_t)(next >> (8 * L)) & 255u;
    next += 1ull << (8 * L);
    const uint32_t rev = __builtin_bitreverse32(c) >> (32 - L);
    for (uint32_t k = 0; k < (1u << (7 - L)); k++) tab[64u * (rev | (k << L)) + (uint32_t)lane] = (uint8_t)(sy | (L << 5));
  }
  const uint32_t total = hlit + hdist;
  uint32_t i = 0, prev = 0, eob = 0, ndist = 0, d1 = 0;
  int lit_left = 32768, dist_left = 32768;
  bool bad = false;
  // straight-line body: every case is computed and selected (lanes decode
  // different candidates, so branches would diverge); a lane that fails
  // stops at the next test of the loop condition
  for (uint32_t it = 0; it < 320u && i < total && !bad; it++) {
    const uint32_t e = tab[64u * (uint32_t)(br.acc & 127u) + (uint32_t)lane];
    const uint32_t sym = e & 31u, cl = e >> 5;
    const uint32_t ex = sym == 16u ? 2u : sym == 17u ? 3u : sym == 18u ? 7u : 0u;
    const uint32_t extra = (uint32_t)(br.acc >> cl) & ((1u << ex) - 1u);
    br.skip(cl + ex);
    const uint32_t L = sym < 16u ? sym : sym == 16u ? prev : 0u;
    const uint32_t rep = sym < 16u ? 1u : (sym == 18u ? 11u : 3u) + extra;
    const uint32_t nl = i < hlit ? min(i + rep, hlit) - i : 0u;
    const uint32_t wgt = L ? 1u << (15u - L) : 0u;  // Kraft weight of one length-L code
    lit_left -= (int)(nl * wgt);
    dist_left -= (int)((rep - nl) * wgt);
    ndist += L ? rep - nl : 0u;
    d1 += L == 1u ? rep - nl : 0u;
    eob = i <= 256u && 256u < i + rep ? L : eob;
    bad = (sym == 16u && i == 0u) || i + rep > total || br.pos > s.end_bits || lit_left < 0 || dist_left < 0;
    prev = L;
    i += rep;
  }
  if (bad || i < total || eob == 0 || lit_left != 0) return false;
  if (dist_left > 0 && ndist != 0 && !(ndist == 1u && d1 == 1u)) return false;
  return true;
}

// Full static check, whole wave: the dynamic tables at b + 3 are valid.
template <bool STORED>
__device__ __forceinline__ bool start_stage2(const Src &s, uint64_t b, TablesLDS &sh, uint32_t mode) {
  if (STORED && (mode & FD_STORED_STARTS) && ((s.peek64(b) >> 1) & 3u) == 0u) return true;  // stored: checked in stage 1
  WaveBits br;
  br.s = s;
  br.init(b + 3);
  return check_dynamic_tables(br, sh) == D_OK;
}

// First candidate in [from, to) that passes the static checks, whole wave.
// *n1 and *n2 (uniform) count the candidates given the table check and the
// ones that passed it.
template <bool STORED>
__device__ __forceinline__ uint64_t wave_find_start(const Src &s, uint64_t from, uint64_t to, TablesLDS &sh,
                                                    uint32_t *n1, uint32_t *n2, uint32_t mode) {
  const int lane = lane_id();
  for (uint64_t b0 = from; b0 < to; b0 += 64) {
    uint64_t b = b0 + (uint64_t)lane;
    bool p = b < to && start_stage1<STORED>(s, b, mode);
    uint64_t m = __ballot(p);
    while (m) {
      int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      (*n1)++;
      if (start_stage2<STORED>(s, b0 + (uint64_t)l, sh, mode)) {
        (*n2)++;
        return b0 + (uint64_t)l;
      }
    }
  }
  return NONE;
}

}  // namespace gzgpu
