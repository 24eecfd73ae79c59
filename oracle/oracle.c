/*
 * CPU oracle for two-pass parallel gzip decompression.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Shares no code
 * with the device path.
 *
 * Format steps follow RFC 1951 (DEFLATE) and RFC 1952 (gzip), which the
 * paper's Section III defers to; the two-pass method follows Section VI-C;
 * block-start detection follows Section VI-A and Appendix A.  Where the paper
 * leaves a point open, the reading taken is stated at the function.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Growable arrays                                                      */
/* ------------------------------------------------------------------ */

static int grow(void **p, size_t *cap, size_t need, size_t elem) {
  if (need <= *cap) return 0;
  size_t c = *cap ? *cap : 4096;
  while (c < need) c *= 2;
  void *q = realloc(*p, c * elem);
  if (!q) return -1;
  *p = q;
  *cap = c;
  return 0;
}

/* ------------------------------------------------------------------ */
/* CRC-32 (RFC 1952 section 8): reflected polynomial 0xEDB88320, register   */
/* preset to all ones, result inverted.  One bit at a time.                */
/* ------------------------------------------------------------------ */

uint32_t orc_crc32(uint32_t crc, const uint8_t *p, size_t n) {
  uint32_t c = crc ^ 0xFFFFFFFFu;
  for (size_t i = 0; i < n; i++) {
    c ^= p[i];
    for (int k = 0; k < 8; k++) c = (c & 1u) ? (c >> 1) ^ 0xEDB88320u : (c >> 1);
  }
  return c ^ 0xFFFFFFFFu;
}

/* ------------------------------------------------------------------ */
/* Bit reader (RFC 1951 section 3.1.1): bits are taken from each byte     */
/* starting with the least significant one.  Reading past the end sets   */
/* the truncation flag and yields zero bits.                              */
/* ------------------------------------------------------------------ */

typedef struct {
  const uint8_t *b;
  size_t n;
  int64_t pos; /* bit position in the whole input */
  int trunc;
} bitrd;

static unsigned get_bit(bitrd *r) {
  size_t byte = (size_t)(r->pos >> 3);
  if (r->pos < 0 || byte >= r->n) {
    r->trunc = 1;
    r->pos++;
    return 0;
  }
  unsigned v = (r->b[byte] >> (r->pos & 7)) & 1u;
  r->pos++;
  return v;
}

/* A multi-bit field: its first bit read is its least significant bit. */
static uint32_t get_bits(bitrd *r, int k) {
  uint32_t v = 0;
  for (int i = 0; i < k; i++) v |= (uint32_t)get_bit(r) << i;
  return v;
}

/* ------------------------------------------------------------------ */
/* Canonical Huffman codes (RFC 1951 section 3.2.2)                     */
/* ------------------------------------------------------------------ */

#define MAXBITS 15

typedef struct {
  int count[MAXBITS + 1];     /* bl_count */
  int next_code[MAXBITS + 1]; /* smallest code of each length */
  int base[MAXBITS + 1];      /* index of the first symbol of each length in sym[] */
  int sym[320];               /* symbols sorted by (code length, symbol value) */
  int ncodes;                 /* symbols with a nonzero length */
  int kraft_left;             /* 2^15 * (1 - sum 2^-len): 0 complete, >0 incomplete, <0 over-subscribed */
} huff;

static void huff_build(huff *h, const uint8_t *len, int n) {
  memset(h, 0, sizeof(*h));
  for (int s = 0; s < n; s++) h->count[len[s]]++;
  h->count[0] = 0;
  for (int s = 0; s < n; s++) h->ncodes += len[s] != 0;
  /* Kraft sum, scaled by 2^15 */
  int left = 1 << MAXBITS;
  for (int L = 1; L <= MAXBITS; L++) left -= h->count[L] << (MAXBITS - L);
  h->kraft_left = left;
  /* step 2 of section 3.2.2: the first code of each length */
  int code = 0;
  for (int L = 1; L <= MAXBITS; L++) {
    code = (code + h->count[L - 1]) << 1;
    h->next_code[L] = code;
  }
  /* step 3: codes of one length go to the symbols in increasing order */
  int b = 0;
  for (int L = 1; L <= MAXBITS; L++) {
    h->base[L] = b;
    b += h->count[L];
  }
  int fill[MAXBITS + 1];
  memcpy(fill, h->base, sizeof(fill));
  for (int s = 0; s < n; s++)
    if (len[s]) h->sym[fill[len[s]]++] = s;
}

/* Huffman codes are packed starting with their most significant bit, so the
 * code grows one bit at a time until it falls in the range of some length. */
static int huff_decode(bitrd *r, const huff *h) {
  int code = 0;
  for (int L = 1; L <= MAXBITS; L++) {
    code = (code << 1) | (int)get_bit(r);
    if (h->count[L] && code >= h->next_code[L] && code < h->next_code[L] + h->count[L])
      return h->sym[h->base[L] + code - h->next_code[L]];
  }
  return -1;
}

/* Lengths and distances (RFC 1951 section 3.2.5). */
static const int len_base[29] = {3,  4,  5,  6,  7,  8,  9,  10, 11,  13,  15,  17,  19,  23, 27,
                                 31, 35, 43, 51, 59, 67, 83, 99, 115, 131, 163, 195, 227, 258};
static const int len_extra[29] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2,
                                  2, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 5, 0};
static const int dist_base[30] = {1,    2,    3,    4,    5,    7,     9,     13,    17,  25,
                                  33,   49,   65,   97,   129,  193,   257,   385,   513, 769,
                                  1025, 1537, 2049, 3073, 4097, 6145, 8193, 12289, 16385, 24577};
static const int dist_extra[30] = {0, 0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6,
                                   6, 7, 7, 8, 8, 9, 9, 10, 10, 11, 11, 12, 12, 13, 13};

/* ------------------------------------------------------------------ */
/* Consumers of decoded literals and matches                            */
/* ------------------------------------------------------------------ */

enum { SINK_BYTES = 0, SINK_SYMBOLS = 1, SINK_CHECK = 2 };

typedef struct {
  int mode;
  /* SINK_BYTES: the plain decompressor.  The history of a member is the
   * member's output so far. */
  uint8_t *out;
  size_t len, cap;
  int64_t *parent;
  size_t parent_cap;
  int want_parent;
  size_t member_start;
  /* SINK_SYMBOLS: decompress(C, w_hat) of Section VI-C */
  uint16_t *sym;
  size_t sym_len, sym_cap;
  int first; /* empty context (the chunk that starts the stream) */
  /* SINK_CHECK: block-start trial decoding, no output kept */
  int64_t check_size;
  int ascii_only;
  int64_t size_cap; /* stop early once the block size reaches this */
} sink;

/* Printable ASCII of the block-start checks: tab, LF, CR and 0x20..0x7E. */
static int is_ascii_text(unsigned c) { return c == 9 || c == 10 || c == 13 || (c >= 32 && c <= 126); }

static int sink_lit(sink *s, unsigned c) {
  switch (s->mode) {
    case SINK_BYTES:
      if (grow((void **)&s->out, &s->cap, s->len + 1, 1)) return -1;
      if (s->want_parent) {
        if (grow((void **)&s->parent, &s->parent_cap, s->len + 1, sizeof(int64_t))) return -1;
        s->parent[s->len] = -1;
      }
      s->out[s->len++] = (uint8_t)c;
      return R_OK;
    case SINK_SYMBOLS:
      if (grow((void **)&s->sym, &s->sym_cap, s->sym_len + 1, 2)) return -1;
      s->sym[s->sym_len++] = (uint16_t)c;
      return R_OK;
    default:
      if (s->ascii_only && !is_ascii_text(c)) return R_NOT_ASCII;
      s->check_size += 1;
      return R_OK;
  }
}

/* A match copies len bytes from dist bytes back, one byte at a time, so a
 * copy that overlaps its own output (dist < len) repeats the pattern. */
static int sink_match(sink *s, int len, int dist) {
  switch (s->mode) {
    case SINK_BYTES: {
      if ((size_t)dist > s->len - s->member_start) return R_TOO_FAR;
      if (grow((void **)&s->out, &s->cap, s->len + len, 1)) return -1;
      if (s->want_parent && grow((void **)&s->parent, &s->parent_cap, s->len + len, sizeof(int64_t)))
        return -1;
      for (int k = 0; k < len; k++) {
        size_t x = s->len;
        s->out[x] = s->out[x - dist];
        if (s->want_parent) s->parent[x] = (int64_t)(x - dist);
        s->len++;
      }
      return R_OK;
    }
    case SINK_SYMBOLS: {
      if (grow((void **)&s->sym, &s->sym_cap, s->sym_len + len, 2)) return -1;
      for (int k = 0; k < len; k++) {
        int64_t src = (int64_t)s->sym_len - dist;
        uint16_t v;
        if (src >= 0) {
          v = s->sym[src];
        } else {
          /* the context w_hat: position src (-32768..-1) holds U_{32768+src} */
          if (s->first) return R_TOO_FAR;
          v = (uint16_t)(0x8000u | (unsigned)(32768 + src));
        }
        s->sym[s->sym_len++] = v;
      }
      return R_OK;
    }
    default:
      /* the context before a candidate block is unknown but always present */
      s->check_size += len;
      return R_OK;
  }
}

/* ------------------------------------------------------------------ */
/* Blocks (RFC 1951 section 3.2.3 .. 3.2.7)                              */
/* ------------------------------------------------------------------ */

/* Dynamic code tables (section 3.2.7).  strict_lit: the literal/length code
 * must be complete (block-start checks); otherwise a lone code of length one
 * is accepted as well. */
static int read_dynamic_tables(bitrd *r, huff *lit, huff *dist, int *no_dist, int strict_lit) {
  static const int order[19] = {16, 17, 18, 0, 8, 7, 9, 6, 10, 5, 11, 4, 12, 3, 13, 2, 14, 1, 15};
  int hlit = (int)get_bits(r, 5) + 257;
  int hdist = (int)get_bits(r, 5) + 1;
  int hclen = (int)get_bits(r, 4) + 4;
  if (r->trunc) return R_TRUNC;
  if (hlit > 286) return R_HLIT;
  if (hdist > 30) return R_HDIST;
  uint8_t cl[19];
  memset(cl, 0, sizeof(cl));
  for (int i = 0; i < hclen; i++) cl[order[i]] = (uint8_t)get_bits(r, 3);
  if (r->trunc) return R_TRUNC;
  huff clh;
  huff_build(&clh, cl, 19);
  if (clh.kraft_left < 0) return R_CL_OVERSUB;
  if (clh.kraft_left > 0) return R_CL_INCOMPLETE;

  uint8_t lens[286 + 30];
  memset(lens, 0, sizeof(lens));
  int total = hlit + hdist;
  int i = 0;
  while (i < total) {
    int sym = huff_decode(r, &clh);
    if (r->trunc) return R_TRUNC;
    if (sym < 0) return R_BAD_CODE;
    if (sym < 16) {
      lens[i++] = (uint8_t)sym;
    } else {
      int rep;
      uint8_t val = 0;
      if (sym == 16) {
        if (i == 0) return R_REPEAT_NO_PREV;
        val = lens[i - 1];
        rep = 3 + (int)get_bits(r, 2);
      } else if (sym == 17) {
        rep = 3 + (int)get_bits(r, 3);
      } else {
        rep = 11 + (int)get_bits(r, 7);
      }
      if (r->trunc) return R_TRUNC;
      if (i + rep > total) return R_REPEAT_OVERRUN;
      while (rep--) lens[i++] = val;
    }
  }
  if (lens[256] == 0) return R_NO_EOB;

  huff_build(lit, lens, hlit);
  if (lit->kraft_left < 0) return R_LIT_OVERSUB;
  if (lit->kraft_left > 0) {
    int lone = lit->ncodes == 1 && lit->count[1] == 1;
    if (strict_lit || !lone) return R_LIT_INCOMPLETE;
  }
  huff_build(dist, lens + hlit, hdist);
  *no_dist = dist->ncodes == 0;
  if (dist->kraft_left < 0) return R_DIST_OVERSUB;
  if (dist->kraft_left > 0 && !*no_dist) {
    int lone = dist->ncodes == 1 && dist->count[1] == 1;
    if (!lone) return R_DIST_INCOMPLETE;
  }
  return R_OK;
}

/* Fixed codes (section 3.2.6). */
static void fixed_tables(huff *lit, huff *dist) {
  uint8_t l[288], d[30];
  int s = 0;
  for (; s < 144; s++) l[s] = 8;
  for (; s < 256; s++) l[s] = 9;
  for (; s < 280; s++) l[s] = 7;
  for (; s < 288; s++) l[s] = 8;
  huff_build(lit, l, 288);
  for (s = 0; s < 30; s++) d[s] = 5;
  huff_build(dist, d, 30);
}

/* Literal/length and distance symbols until end-of-block (section 3.2.5).
 * For the fixed code the distance codes 30 and 31 are also 5 bits long; they
 * are not in the table and land on the "no symbol" path after 5 bits. */
static int decode_codes(bitrd *r, const huff *lit, const huff *dist, int no_dist, int fixed, sink *s,
                        int64_t *nsym) {
  for (;;) {
    int sym = huff_decode(r, lit);
    if (r->trunc) return R_TRUNC;
    if (sym < 0) return R_BAD_CODE;
    (*nsym)++;
    if (sym < 256) {
      int e = sink_lit(s, (unsigned)sym);
      if (e) return e;
    } else if (sym == 256) {
      return R_OK;
    } else {
      if (sym > 285) return R_BAD_LITLEN;
      int len = len_base[sym - 257] + (int)get_bits(r, len_extra[sym - 257]);
      if (no_dist) return R_NO_DIST;
      int dsym;
      if (fixed) {
        /* fixed distance codes are the 5-bit values 0..31 written MSB first */
        dsym = 0;
        for (int k = 0; k < 5; k++) dsym = (dsym << 1) | (int)get_bit(r);
      } else {
        dsym = huff_decode(r, dist);
      }
      if (r->trunc) return R_TRUNC;
      if (dsym < 0) return R_BAD_CODE;
      if (dsym > 29) return R_BAD_DIST;
      int d = dist_base[dsym] + (int)get_bits(r, dist_extra[dsym]);
      if (r->trunc) return R_TRUNC;
      int e = sink_match(s, len, d);
      if (e) return e;
    }
    if (s->mode == SINK_CHECK && s->check_size >= s->size_cap) return R_SIZE;
  }
}

/* One block: header, then its body. */
static int inflate_block(bitrd *r, sink *s, int *bfinal, int *btype, int64_t *nsym, int strict_lit) {
  *bfinal = (int)get_bit(r);
  *btype = (int)get_bits(r, 2);
  if (r->trunc) return R_TRUNC;
  if (*btype == 3) return R_BTYPE3;
  if (*btype == 0) {
    /* stored: skip to a byte boundary, LEN, NLEN, then LEN raw bytes */
    r->pos = (r->pos + 7) & ~(int64_t)7;
    uint32_t len = get_bits(r, 16);
    uint32_t nlen = get_bits(r, 16);
    if (r->trunc) return R_TRUNC;
    if ((len ^ 0xFFFFu) != nlen) return R_NLEN;
    for (uint32_t k = 0; k < len; k++) {
      unsigned c = get_bits(r, 8);
      if (r->trunc) return R_TRUNC;
      int e = sink_lit(s, c);
      if (e) return e;
    }
    return R_OK;
  }
  huff lit, dist;
  int no_dist = 0;
  if (*btype == 1) {
    fixed_tables(&lit, &dist);
  } else {
    int e = read_dynamic_tables(r, &lit, &dist, &no_dist, strict_lit);
    if (e) return e;
  }
  return decode_codes(r, &lit, &dist, no_dist, *btype == 1, s, nsym);
}

static int reason_status(int reason) {
  switch (reason) {
    case R_OK: return ORC_OK;
    case R_MAGIC: case R_CM: case R_FLG: case R_HCRC: case R_GARBAGE: return ORC_E_HEADER;
    case R_CRC: return ORC_E_CRC;
    case R_ISIZE: return ORC_E_SIZE;
    case -1: return ORC_E_MEM;
    default: return ORC_E_DATA;
  }
}

/* ------------------------------------------------------------------ */
/* gzip member header (RFC 1952 section 2.3)                             */
/* ------------------------------------------------------------------ */

int orc_parse_header(const uint8_t *in, size_t n, size_t *payload_start, int *reason) {
  size_t p = 0;
  *reason = R_OK;
  if (n < 10) { *reason = R_TRUNC; return ORC_E_HEADER; }
  if (in[0] != 0x1f || in[1] != 0x8b) { *reason = R_MAGIC; return ORC_E_HEADER; }
  if (in[2] != 8) { *reason = R_CM; return ORC_E_HEADER; }
  unsigned flg = in[3];
  if (flg & 0xE0) { *reason = R_FLG; return ORC_E_HEADER; }
  p = 10; /* ID1 ID2 CM FLG MTIME(4) XFL OS */
  if (flg & 4) { /* FEXTRA */
    if (p + 2 > n) { *reason = R_TRUNC; return ORC_E_HEADER; }
    size_t xlen = (size_t)in[p] | ((size_t)in[p + 1] << 8);
    p += 2 + xlen;
    if (p > n) { *reason = R_TRUNC; return ORC_E_HEADER; }
  }
  if (flg & 8) { /* FNAME, zero-terminated */
    while (p < n && in[p]) p++;
    if (p >= n) { *reason = R_TRUNC; return ORC_E_HEADER; }
    p++;
  }
  if (flg & 16) { /* FCOMMENT, zero-terminated */
    while (p < n && in[p]) p++;
    if (p >= n) { *reason = R_TRUNC; return ORC_E_HEADER; }
    p++;
  }
  if (flg & 2) { /* FHCRC: low 16 bits of the CRC-32 of the header so far */
    if (p + 2 > n) { *reason = R_TRUNC; return ORC_E_HEADER; }
    uint32_t want = (uint32_t)in[p] | ((uint32_t)in[p + 1] << 8);
    if ((orc_crc32(0, in, p) & 0xFFFFu) != want) { *reason = R_HCRC; return ORC_E_HEADER; }
    p += 2;
  }
  *payload_start = p;
  return ORC_OK;
}

static uint32_t rd32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

/* ------------------------------------------------------------------ */
/* Sequential gunzip: every member, blocks in order, CRC-32 and ISIZE     */
/* checked against each trailer.                                          */
/* ------------------------------------------------------------------ */

orc_gunzip_result *orc_gunzip(const uint8_t *in, size_t n, int want_parent) {
  orc_gunzip_result *res = (orc_gunzip_result *)calloc(1, sizeof(*res));
  if (!res) return NULL;
  sink s;
  memset(&s, 0, sizeof(s));
  s.mode = SINK_BYTES;
  s.want_parent = want_parent;
  size_t blocks_cap = 0;
  size_t p = 0;
  int reason = R_OK;
  int member = 0;
  while (p < n) {
    size_t h;
    int hr;
    if (orc_parse_header(in + p, n - p, &h, &hr) != ORC_OK) {
      reason = member == 0 ? hr : R_GARBAGE;
      break;
    }
    h += p;
    if (member == 0) res->payload_start = h;
    s.member_start = s.len;
    bitrd r = {in, n, (int64_t)h * 8, 0};
    int bfinal = 0;
    while (!bfinal) {
      if (grow((void **)&res->blocks, &blocks_cap, res->n_blocks + 1, sizeof(orc_block))) { reason = -1; break; }
      orc_block *b = &res->blocks[res->n_blocks];
      memset(b, 0, sizeof(*b));
      b->bit = r.pos;
      b->out_off = (int64_t)s.len;
      b->member = member;
      int btype = 0;
      int64_t nsym = 0;
      int e = inflate_block(&r, &s, &bfinal, &btype, &nsym, 0);
      b->btype = btype;
      b->bfinal = bfinal;
      b->nsym = nsym;
      b->out_len = (int64_t)s.len - b->out_off;
      res->n_blocks++;
      if (e) { reason = e; break; }
    }
    if (reason) break;
    /* the trailer starts at the next byte boundary */
    int64_t endbit = r.pos;
    size_t t = (size_t)((r.pos + 7) >> 3);
    if (t + 8 > n) { reason = R_TRUNC; break; }
    uint32_t crc = rd32(in + t), isz = rd32(in + t + 4);
    uint32_t mine = orc_crc32(0, s.out + s.member_start, s.len - s.member_start);
    if (member == 0) {
      res->end_bit = endbit;
      res->trailer_at = t;
      res->crc_trailer = crc;
      res->isize_trailer = isz;
      res->crc_computed = mine;
    }
    member++;
    if (crc != mine) { reason = R_CRC; break; }
    if (isz != (uint32_t)((s.len - s.member_start) & 0xFFFFFFFFu)) { reason = R_ISIZE; break; }
    p = t + 8;
  }
  res->n_members = member;
  res->reason = reason;
  res->status = reason_status(reason);
  res->out = s.out;
  res->out_len = s.len;
  res->parent = s.parent;
  return res;
}

void orc_gunzip_free(orc_gunzip_result *r) {
  if (!r) return;
  free(r->out);
  free(r->parent);
  free(r->blocks);
  free(r);
}

/* ------------------------------------------------------------------ */
/* Pass 1: decompress(C_i, w_hat_i) of Section VI-C                     */
/* ------------------------------------------------------------------ */

orc_sym_result *orc_symbolic(const uint8_t *in, size_t n, int64_t start_bit, int64_t stop_bit, int first) {
  orc_sym_result *res = (orc_sym_result *)calloc(1, sizeof(*res));
  if (!res) return NULL;
  sink s;
  memset(&s, 0, sizeof(s));
  s.mode = SINK_SYMBOLS;
  s.first = first;
  bitrd r = {in, n, start_bit, 0};
  int reason = R_OK;
  size_t bits_cap = 0;
  for (;;) {
    /* stop before the first block that starts at or after the stop bit */
    if (r.pos >= stop_bit) break;
    /* where each block header begins (RFC 1951 section 3.2.3), as in orc_gunzip's block map */
    if (grow((void **)&res->block_bits, &bits_cap, (size_t)res->n_blocks + 1, sizeof(int64_t))) {
      reason = -1;
      break;
    }
    res->block_bits[res->n_blocks] = r.pos;
    int bfinal = 0, btype = 0;
    int64_t nsym = 0;
    int e = inflate_block(&r, &s, &bfinal, &btype, &nsym, 0);
    res->n_syms += nsym;
    res->n_blocks++;
    if (e) { reason = e; break; }
    if (bfinal) { res->final_reached = 1; break; }
  }
  res->end_bit = r.pos;
  res->reason = reason;
  res->status = reason_status(reason);
  res->sym = s.sym;
  res->len = s.sym_len;
  for (size_t i = 0; i < s.sym_len; i++) res->n_placeholders += s.sym[i] >= 0x8000;
  return res;
}

void orc_sym_free(orc_sym_result *r) {
  if (!r) return;
  free(r->sym);
  free(r->block_bits);
  free(r);
}

/* ------------------------------------------------------------------ */
/* Block-start checks (Section VI-A, Appendix A)                         */
/*                                                                        */
/* Readings taken where the paper gives no detail:                        */
/*  - a chunk may only start on a dynamic-Huffman block (BTYPE 10);       */
/*  - "invalid Huffman tree": HLIT <= 286, HDIST <= 30, complete code-    */
/*    length code, no repeat before the first length, no repeat past the  */
/*    end, end-of-block present, complete literal/length code, distance   */
/*    code complete or a lone one-bit code or empty;                      */
/*  - "valid ASCII": tab, LF, CR and 0x20..0x7E;                          */
/*  - "larger than 1 KiB and smaller than 4 MiB": 1024 < size < 4194304   */
/*    bytes produced by the candidate block;                              */
/*  - "decompress five more blocks": each has a valid header and codes    */
/*    and ASCII literals; a final block ends the check successfully.      */
/* ------------------------------------------------------------------ */

#define CONFIRM_BLOCKS 5
#define MIN_BLOCK 1024
#define MAX_BLOCK (4 << 20)

int orc_block_static(const uint8_t *in, size_t n, int64_t bit, int *reason) {
  return orc_block_static_types(in, n, bit, ORC_START_DYNAMIC, reason);
}

/* Start types (a reading of Appendix A, which rejects only BTYPE 11): a
 * stored block is a candidate when its padding bits are zero, LEN and NLEN
 * are complements and LEN > 1 KiB (the trial block's size bound); a fixed
 * block has no table to check, so the trial block is its only test. */
int orc_block_static_types(const uint8_t *in, size_t n, int64_t bit, int types, int *reason) {
  bitrd r = {in, n, bit, 0};
  int bfinal = (int)get_bit(&r);
  int btype = (int)get_bits(&r, 2);
  int e = R_OK;
  if (r.trunc) e = R_TRUNC;
  else if (bfinal) e = R_FINAL;
  else if (btype == 0 && (types & ORC_START_STORED)) {
    int64_t p = (bit + 3 + 7) & ~(int64_t)7;
    while (r.pos < p && !r.trunc && !e)
      if (get_bit(&r)) e = R_NOT_DYNAMIC;
    uint32_t len = get_bits(&r, 16), nlen = get_bits(&r, 16);
    if (!e && r.trunc) e = R_TRUNC;
    else if (!e && (len ^ 0xFFFFu) != nlen) e = R_NLEN;
    else if (!e && len <= MIN_BLOCK) e = R_SIZE;
  } else if (btype == 1 && (types & ORC_START_FIXED)) {
    e = R_OK;
  } else if (btype != 2) e = R_NOT_DYNAMIC;
  else {
    huff lit, dist;
    int no_dist;
    e = read_dynamic_tables(&r, &lit, &dist, &no_dist, 1);
  }
  if (reason) *reason = e;
  return e == R_OK;
}

int orc_block_predicate(const uint8_t *in, size_t n, int64_t bit, int *reason) {
  return orc_block_predicate_types(in, n, bit, 1, ORC_START_DYNAMIC, reason);
}

int orc_block_predicate_mode(const uint8_t *in, size_t n, int64_t bit, int ascii, int *reason) {
  return orc_block_predicate_types(in, n, bit, ascii, ORC_START_DYNAMIC, reason);
}

/* Binary inputs (Section VIII lists them as a limitation): the same checks
 * without the ASCII test of the literals. */
int orc_block_predicate_types(const uint8_t *in, size_t n, int64_t bit, int ascii, int types, int *reason) {
  int e;
  if (!orc_block_static_types(in, n, bit, types, &e)) {
    if (reason) *reason = e;
    return 0;
  }
  sink s;
  memset(&s, 0, sizeof(s));
  s.mode = SINK_CHECK;
  s.ascii_only = ascii;
  s.size_cap = MAX_BLOCK;
  bitrd r = {in, n, bit, 0};
  int bfinal, btype;
  int64_t nsym = 0;
  e = inflate_block(&r, &s, &bfinal, &btype, &nsym, 1);
  if (!e && !(s.check_size > MIN_BLOCK && s.check_size < MAX_BLOCK)) e = R_SIZE;
  for (int k = 0; !e && k < CONFIRM_BLOCKS; k++) {
    s.check_size = 0;
    s.size_cap = INT64_MAX;
    e = inflate_block(&r, &s, &bfinal, &btype, &nsym, 0);
    if (!e && bfinal) break;
  }
  if (reason) *reason = e;
  return e == R_OK;
}

int64_t orc_find_start(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only) {
  return orc_find_start_mode(in, n, lo, hi, static_only, 1);
}

int64_t orc_find_start_mode(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only, int ascii) {
  return orc_find_start_types(in, n, lo, hi, static_only, ascii, ORC_START_DYNAMIC);
}

int64_t orc_find_start_types(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only, int ascii,
                             int types) {
  for (int64_t b = lo; b < hi; b++) {
    int ok = static_only ? orc_block_static_types(in, n, b, types, NULL)
                         : orc_block_predicate_types(in, n, b, ascii, types, NULL);
    if (ok) return b;
  }
  return -1;
}

/* ------------------------------------------------------------------ */
/* The two-pass method (Section VI-C)                                     */
/* ------------------------------------------------------------------ */

void orc_pugz_free(orc_pugz_result *r) {
  if (!r) return;
  free(r->nominal);
  free(r->start);
  free(r->cand);
  free(r->end);
  free(r->len);
  free(r->off);
  free(r->placeholders);
  free(r->valid);
  free(r->windows);
  free(r->out);
  free(r);
}

orc_pugz_result *orc_pugz(const uint8_t *in, size_t n, int N) { return orc_pugz_types(in, n, N, 1, ORC_START_DYNAMIC); }

orc_pugz_result *orc_pugz_mode(const uint8_t *in, size_t n, int N, int ascii) {
  return orc_pugz_types(in, n, N, ascii, ORC_START_DYNAMIC);
}

/* A chunk that starts on a stored header, at s, and a previous chunk that
 * ended at e with s < e in the same run of zero bits before the same
 * LEN/NLEN: both bits begin the same stored block, so decoding from either
 * gives the same symbols and the same end. */
static int stored_equivalent(const uint8_t *in, size_t n, int64_t s, int64_t e, int types) {
  if (!(types & ORC_START_STORED) || !(s < e)) return 0;
  if (((s + 3 + 7) >> 3) != ((e + 3 + 7) >> 3)) return 0;
  bitrd r = {in, n, s, 0};
  if (get_bits(&r, 3) != 0 || r.trunc) return 0;
  return orc_block_static_types(in, n, s, ORC_START_STORED, NULL);
}

orc_pugz_result *orc_pugz_types(const uint8_t *in, size_t n, int N, int ascii, int types) {
  orc_pugz_result *res = (orc_pugz_result *)calloc(1, sizeof(*res));
  if (!res || N < 1) return res;
  res->n_chunks = N;
  res->nominal = (int64_t *)calloc((size_t)N + 1, 8);
  res->start = (int64_t *)calloc((size_t)N, 8);
  res->cand = (int64_t *)calloc((size_t)N, 8);
  res->end = (int64_t *)calloc((size_t)N, 8);
  res->len = (int64_t *)calloc((size_t)N, 8);
  res->off = (int64_t *)calloc((size_t)N, 8);
  res->placeholders = (int64_t *)calloc((size_t)N, 8);
  res->valid = (int64_t *)calloc((size_t)N, 8);
  res->windows = (uint8_t *)calloc((size_t)N, 32768);
  orc_sym_result **D = (orc_sym_result **)calloc((size_t)N, sizeof(*D));
  if (!res->nominal || !res->start || !res->cand || !res->end || !res->len || !res->off ||
      !res->placeholders || !res->valid || !res->windows || !D) {
    res->status = ORC_E_MEM;
    free(D);
    return res;
  }
  int reason = R_OK;
  size_t h;
  if (orc_parse_header(in, n, &h, &reason) != ORC_OK || n < h + 8) {
    res->reason = reason ? reason : R_TRUNC;
    res->status = ORC_E_HEADER;
    free(D);
    return res;
  }
  res->crc_trailer = rd32(in + n - 8);
  res->isize_trailer = rd32(in + n - 4);

  /* split the payload into N roughly equal compressed parts */
  int64_t P = (int64_t)(n - 8 - h);
  for (int i = 0; i <= N; i++) res->nominal[i] = (int64_t)h + (int64_t)((__int128)i * P / N);

  /* block starts: chunk 0 at the payload's first bit, others searched */
  res->start[0] = res->cand[0] = (int64_t)h * 8;
  for (int i = 1; i < N; i++) {
    res->cand[i] = orc_find_start_types(in, n, res->nominal[i] * 8, res->nominal[i + 1] * 8, 0, ascii, types);
    res->start[i] = res->cand[i];
  }

  /* pass 1, chunk by chunk, each stopping at the next non-empty chunk's start;
   * a start the previous chunk does not end on is replaced by that end */
  int prev = -1;
  int final_seen = 0;
  for (int i = 0; i < N; i++) {
    res->end[i] = -1;
    if (res->start[i] < 0) continue;
    if (final_seen) { res->start[i] = -1; continue; }
    if (prev >= 0 && res->end[prev] != res->start[i]) {
      if (stored_equivalent(in, n, res->start[i], res->end[prev], types)) res->n_equivalent++;
      else res->n_repairs++;
      res->start[i] = res->end[prev];
    }
    int64_t stop = INT64_MAX;
    for (int j = i + 1; j < N; j++)
      if (res->start[j] >= 0) { stop = res->start[j]; break; }
    if (res->start[i] >= stop) {
      /* the previous chunk already decoded past this one */
      res->end[i] = res->start[i];
      res->len[i] = 0;
      D[i] = (orc_sym_result *)calloc(1, sizeof(orc_sym_result));
      D[i]->end_bit = res->start[i];
      prev = i;
      continue;
    }
    D[i] = orc_symbolic(in, n, res->start[i], stop, i == 0);
    if (!D[i]) { reason = -1; break; }
    if (D[i]->status != ORC_OK) { reason = D[i]->reason; break; }
    res->end[i] = D[i]->end_bit;
    res->len[i] = (int64_t)D[i]->len;
    res->placeholders[i] = D[i]->n_placeholders;
    if (D[i]->final_reached) final_seen = 1;
    prev = i;
  }
  if (!reason && !final_seen) reason = R_TRUNC;
  if (!reason) {
    /* the stream must end exactly where the trailer starts */
    int64_t endbit = res->end[prev];
    if ((size_t)((endbit + 7) >> 3) + 8 != n) reason = R_GARBAGE;
  }

  /* pass 2: windows resolved in chunk order.  w_next = the last 32768
   * symbols of (w_hat_i ++ D_i), each U_j replaced by w_i[j].  valid counts
   * the real bytes of history, so window entries before the data start stay
   * unknown (zero). */
  int64_t off = 0;
  uint8_t *w = NULL;
  int64_t valid = 0;
  if (!reason) {
    for (int i = 0; i < N; i++) {
      res->off[i] = off;
      res->valid[i] = valid;
      if (res->start[i] < 0) continue;
      if (w) memcpy(res->windows + (size_t)i * 32768, w, 32768);
      uint8_t *wi = res->windows + (size_t)i * 32768;
      uint8_t *wn = (uint8_t *)malloc(32768);
      if (!wn) { reason = -1; break; }
      int64_t L = res->len[i];
      for (int64_t k = 0; k < 32768; k++) {
        int64_t q = L + k; /* index into w_hat_i ++ D_i */
        uint16_t t = q < 32768 ? (uint16_t)(0x8000u | (unsigned)q) : D[i]->sym[q - 32768];
        wn[k] = t < 256 ? (uint8_t)t : wi[t & 0x7FFF];
      }
      free(w);
      w = wn;
      off += L;
      valid = valid + L > 32768 ? 32768 : valid + L;
    }
    free(w);
  }

  /* translation: U_j in D_i becomes w_i[j]; a U_j that lies before the data
   * start is a distance reaching too far back */
  if (!reason) {
    res->out_len = (size_t)off;
    res->out = (uint8_t *)malloc(res->out_len ? res->out_len : 1);
    if (!res->out) reason = -1;
    for (int i = 0; !reason && i < N; i++) {
      if (res->start[i] < 0) continue;
      const uint8_t *wi = res->windows + (size_t)i * 32768;
      for (int64_t p = 0; p < res->len[i]; p++) {
        uint16_t t = D[i]->sym[p];
        if (t < 256) {
          res->out[res->off[i] + p] = (uint8_t)t;
        } else {
          unsigned j = t & 0x7FFF;
          if ((int64_t)j < 32768 - res->valid[i]) { reason = R_TOO_FAR; break; }
          res->out[res->off[i] + p] = wi[j];
        }
      }
    }
  }
  if (!reason) {
    res->crc_computed = orc_crc32(0, res->out, res->out_len);
    if (res->crc_computed != res->crc_trailer) reason = R_CRC;
    else if ((uint32_t)(res->out_len & 0xFFFFFFFFu) != res->isize_trailer) reason = R_ISIZE;
  }
  for (int i = 0; i < N; i++) orc_sym_free(D[i]);
  free(D);
  res->reason = reason;
  res->status = reason == R_GARBAGE ? ORC_E_UNSUPPORTED : reason_status(reason);
  return res;
}
