/*
 * CPU oracle for two-pass parallel gzip decompression.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, sequential C written from the
 * DEFLATE and gzip format definitions (RFC 1951, RFC 1952; the paper defers
 * the format to them in Section III) and from the paper's description of the
 * two-pass method (Section VI-C) and of block-start detection (Section VI-A,
 * Appendix A).  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code with the device
 * path.
 *
 * Bits are read one at a time, Huffman codes are decoded one bit at a time
 * against the canonical code of RFC 1951 section 3.2.2, and match copies go
 * byte by byte, so each step can be checked against the RFC by eye.
 */
#ifndef GZ_ORACLE_H
#define GZ_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  ORC_OK = 0,
  ORC_E_HEADER = -2,      /* gzip member header invalid */
  ORC_E_UNSUPPORTED = -3, /* more than one member where only one is handled */
  ORC_E_DATA = -4,        /* invalid DEFLATE data */
  ORC_E_CRC = -6,         /* trailer CRC-32 mismatch */
  ORC_E_SIZE = -7,        /* trailer ISIZE mismatch */
  ORC_E_MEM = -8
};

/* finer reasons (the status is derived from them) */
enum {
  R_OK = 0,
  R_TRUNC = 1,          /* ran past the end of the input */
  R_BTYPE3 = 2,         /* reserved block type 11 */
  R_NLEN = 3,           /* stored block NLEN != ~LEN */
  R_HLIT = 4,           /* more than 286 literal/length codes */
  R_HDIST = 5,          /* more than 30 distance codes */
  R_CL_OVERSUB = 6,
  R_CL_INCOMPLETE = 7,
  R_REPEAT_NO_PREV = 8, /* code 16 with no previous length */
  R_REPEAT_OVERRUN = 9, /* repeat runs past HLIT+HDIST */
  R_NO_EOB = 10,        /* end-of-block symbol has no code */
  R_LIT_OVERSUB = 11,
  R_LIT_INCOMPLETE = 12,
  R_DIST_OVERSUB = 13,
  R_DIST_INCOMPLETE = 14,
  R_BAD_CODE = 15,      /* bit pattern of an incomplete code with no symbol */
  R_BAD_LITLEN = 16,    /* literal/length symbol 286 or 287 */
  R_BAD_DIST = 17,      /* distance symbol 30 or 31 */
  R_NO_DIST = 18,       /* a match in a block that has no distance codes */
  R_TOO_FAR = 19,       /* distance reaches before the start of the data */
  R_MAGIC = 20,
  R_CM = 21,
  R_FLG = 22,
  R_HCRC = 23,
  R_CRC = 24,
  R_ISIZE = 25,
  R_GARBAGE = 26,       /* bytes after a member that do not start a member */
  R_NOT_ASCII = 27,     /* block-start checks: literal outside the ASCII set */
  R_SIZE = 28,          /* block-start checks: block size out of bounds */
  R_NOT_DYNAMIC = 29,   /* block-start checks: candidate not BTYPE 10 */
  R_FINAL = 30          /* block-start checks: candidate has BFINAL set */
};

typedef struct {
  int64_t bit;      /* bit offset of the block header in the whole input */
  int32_t btype;    /* 0 stored, 1 fixed, 2 dynamic */
  int32_t bfinal;
  int64_t out_off;  /* output offset of the block's first byte */
  int64_t out_len;  /* bytes the block produces */
  int64_t nsym;     /* Huffman literal/length symbols decoded, end-of-block included */
  int32_t member;
  int32_t pad;
} orc_block;

typedef struct {
  int status;       /* ORC_* */
  int reason;       /* R_* */
  uint8_t *out;
  size_t out_len;
  int64_t *parent;  /* per output byte: x - d for match bytes, -1 otherwise; NULL unless asked */
  orc_block *blocks;
  size_t n_blocks;
  int n_members;
  size_t payload_start;  /* first member: byte where DEFLATE data begins */
  int64_t end_bit;       /* first member: bit after its final block */
  size_t trailer_at;     /* first member: byte offset of its trailer */
  uint32_t crc_trailer;  /* first member */
  uint32_t isize_trailer;
  uint32_t crc_computed;
} orc_gunzip_result;

/* Sequential gunzip of every member (RFC 1952 section 2.2). */
orc_gunzip_result *orc_gunzip(const uint8_t *in, size_t n, int want_parent);
void orc_gunzip_free(orc_gunzip_result *r);

/* gzip member header: returns ORC_OK and the byte where DEFLATE data begins. */
int orc_parse_header(const uint8_t *in, size_t n, size_t *payload_start, int *reason);

/* CRC-32 of RFC 1952 section 8 (reflected 0xEDB88320, pre/post inversion). */
uint32_t orc_crc32(uint32_t crc, const uint8_t *p, size_t n);

/* Pass 1 of the two-pass method: decompress(C_i, w_hat_i).
 * Decodes whole blocks from start_bit and stops before the first block header
 * whose bit offset is >= stop_bit, or after a final block.  With first != 0
 * the context is empty (the chunk that starts the stream); otherwise it is
 * 32768 unique symbols U_j, written 0x8000 | j, U_32767 being the byte just
 * before the chunk.  Output symbols are 0..255 for bytes and 0x8000|j for U_j. */
typedef struct {
  int status;
  int reason;
  uint16_t *sym;
  size_t len;
  int64_t end_bit;        /* e: where decoding stopped */
  int final_reached;
  int64_t n_blocks;
  int64_t n_syms;         /* Huffman literal/length symbols, end-of-block included */
  int64_t n_placeholders; /* output symbols >= 0x8000 */
  int64_t *block_bits;    /* bit offset of every block header decoded, in order (n_blocks entries) */
} orc_sym_result;

orc_sym_result *orc_symbolic(const uint8_t *in, size_t n, int64_t start_bit, int64_t stop_bit, int first);
void orc_sym_free(orc_sym_result *r);

/* Block-start checks of Appendix A.
 * orc_block_static: BFINAL = 0, BTYPE = 10 and valid code tables at bit b.
 * orc_block_predicate: the static checks, then the block decodes with
 * printable-ASCII literals and 1024 < size < 4 MiB, then five more blocks
 * decode with valid headers and codes and ASCII literals (a final block ends
 * the confirmation with success).  Returns 1 or 0; *stage gets the failing
 * reason (R_*) or R_OK. */
int orc_block_static(const uint8_t *in, size_t n, int64_t bit, int *reason);
/* Block types accepted as chunk starts (a mask; dynamic is always on). */
#define ORC_START_DYNAMIC 1
#define ORC_START_STORED 2
#define ORC_START_FIXED 4
int orc_block_static_types(const uint8_t *in, size_t n, int64_t bit, int types, int *reason);
int orc_block_predicate(const uint8_t *in, size_t n, int64_t bit, int *reason);
/* ascii 0: binary inputs, the same checks without the ASCII test. */
int orc_block_predicate_mode(const uint8_t *in, size_t n, int64_t bit, int ascii, int *reason);
int orc_block_predicate_types(const uint8_t *in, size_t n, int64_t bit, int ascii, int types, int *reason);
/* Smallest b in [lo, hi) passing the predicate (static only if static_only), or -1. */
int64_t orc_find_start(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only);
int64_t orc_find_start_mode(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only, int ascii);
int64_t orc_find_start_types(const uint8_t *in, size_t n, int64_t lo, int64_t hi, int static_only, int ascii,
                             int types);

/* The whole two-pass method of Section VI-C on the CPU, single member.
 * Chunk i covers compressed bytes [nom_i, nom_{i+1}) of the payload with
 * nom_i = h + floor(i * P / N); chunk 0 starts at the payload's first bit,
 * chunk i >= 1 at the first bit of its range passing orc_block_predicate
 * (none: the chunk is empty).  Pass 1 decodes each chunk up to the next
 * non-empty chunk's start; a start that the previous chunk does not end on
 * is replaced by that chunk's end and decoded again.  Pass 2 resolves the
 * windows in chunk order and replaces every U_j. */
typedef struct {
  int status;
  int reason;
  int n_chunks;
  int64_t *nominal;       /* n_chunks + 1 byte offsets */
  int64_t *start;         /* final start bit, -1 for an empty chunk */
  int64_t *cand;          /* start found by the block-start search, -1 if none */
  int64_t *end;           /* e_i, -1 for an empty chunk */
  int64_t *len;           /* |D_i| */
  int64_t *off;           /* output offset of chunk i */
  int64_t *placeholders;  /* symbols >= 0x8000 in D_i */
  int64_t *valid;         /* real history bytes before chunk i, capped at 32768 */
  uint8_t *windows;       /* n_chunks * 32768: resolved window before chunk i */
  int n_repairs;
  int n_equivalent;       /* stored starts taken as the previous chunk's end (same block) */
  uint8_t *out;
  size_t out_len;
  uint32_t crc_trailer, isize_trailer, crc_computed;
} orc_pugz_result;

orc_pugz_result *orc_pugz(const uint8_t *in, size_t n, int n_chunks);
/* ascii 0: the block-start search of binary inputs (no ASCII test). */
orc_pugz_result *orc_pugz_mode(const uint8_t *in, size_t n, int n_chunks, int ascii);
/* types: also stored and/or fixed blocks as chunk starts.  A stored start
 * that the previous chunk's end reaches in the same zero run before the same
 * LEN/NLEN is taken as that end without a repair (n_equivalent). */
orc_pugz_result *orc_pugz_types(const uint8_t *in, size_t n, int n_chunks, int ascii, int types);
void orc_pugz_free(orc_pugz_result *r);

#ifdef __cplusplus
}
#endif
#endif
