/*
 * gzgpu: two-pass parallel gzip decompression on one AMD Instinct MI355X.
 *
 * The method is the one of Kerbiriou & Chikhi, "Parallel decompression of
 * gzip-compressed files and random access to DNA sequences", Section VI-C:
 * the compressed payload of one gzip member is cut into parts; each part
 * finds a DEFLATE block start (Section VI-A, Appendix A), decodes with a
 * context of 32768 unique placeholder symbols (pass 1), the 32 KiB windows
 * are resolved part after part, and every placeholder is replaced by its
 * byte (pass 2).  The output is the exact gunzip of the member.
 *
 * Memory model
 *   - Every buffer handed to these calls is HIP device memory owned by the
 *     caller: compressed input, output, workspace, and a server's arena.
 *     The library allocates no device memory; it keeps a small pinned host
 *     copy of each plan's job table, and a stream a 32 KiB pinned host
 *     buffer for its carried window.
 *   - The compressed input must stay alive and unmodified until the stream
 *     work of a gz_decompress* call has completed.
 *   - A plan is used by one stream at a time.  Distinct plans (with distinct
 *     workspaces) are independent.
 *
 * Errors
 *   - Every call returns an int: GZ_OK (0) or a negative GZ_E_* code; nothing
 *     is thrown across this interface.  gz_strerror() gives a message.
 *   - gz_decompress* only enqueues work.  Data errors are reported by
 *     gz_result*, which waits for the stream.
 */
#ifndef GZGPU_H
#define GZGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GZ_OK 0
#define GZ_E_ARG (-1)         /* invalid argument (NULL, size 0, bad options) */
#define GZ_E_HEADER (-2)      /* gzip member header invalid (magic, CM, reserved FLG bits, FHCRC) */
#define GZ_E_UNSUPPORTED (-3) /* bytes after the first member (multi-member input) */
#define GZ_E_DATA (-4)        /* invalid DEFLATE data, truncation, distance too far back */
#define GZ_E_CAPACITY (-5)    /* output or workspace too small; gz_result gives the sizes needed */
#define GZ_E_CRC (-6)         /* CRC-32 of the output differs from the trailer's (RFC 1952 section 8) */
#define GZ_E_SIZE (-7)        /* CRC matches but the length differs from the trailer's ISIZE (mod 2^32) */
#define GZ_E_HIP (-9)         /* HIP runtime error */
#define GZ_E_NOT_READY (-10)  /* gz_result before any gz_decompress on this plan */

#define GZ_START_STORED 2u

/* Options.  An all-zero struct means defaults.  (Section VI-C cuts the payload
 * into n roughly equal parts; Section VI-A and Appendix A give the
 * block-start checks whose constants appear here.) */
typedef struct gz_opts {
  uint64_t chunk_bytes;   /* nominal compressed bytes per chunk when n_chunks == 0 (default 40 KiB) */
  uint32_t sym_factor;    /* symbol capacity per chunk = sym_factor * compressed bytes + slack (default 8) */
  uint32_t window_syms;   /* LDS history ring per decoding wave, in symbols: 512, 1024, 2048, 4096, 8192, 16384
                             or 32768 (default 512); match sources further back are read from HBM.
                             Any other value: GZ_E_ARG */
  uint32_t scan_groups;   /* workgroups that search one chunk's start in parallel (default: 4096 / chunks, 1..64) */
  uint32_t inflate_waves_per_cu; /* persistent inflate grid = this * CU count (default: occupancy) */
  uint32_t waves_per_chunk; /* each nominal chunk is split into this many sub-chunks, one wave each (default 1) */
  uint32_t timing;        /* nonzero: record a HIP event at every pass boundary (see gz_pass_times) */
  uint32_t confirm_decode; /* nonzero: confirmation blocks a chunk owes past its stop are always decoded
                              on their own instead of taken from the next chunks (same result; tests) */
  uint32_t binary;        /* nonzero: binary input (Section VIII): chunk starts are searched with the checks
                             of Appendix A except the ASCII test of the literals; the output is exact
                             either way (the stitch check repairs any wrong start) */
  uint32_t tuned;         /* nonzero: a file whose (compressed-size, ratio) class gz_autotune has timed on this
                             device takes the chunk size chosen there (over chunk_bytes), and, unless
                             window_syms is set, the plan takes the ring chosen for its largest such file */
  uint32_t start_types;   /* block types searched as chunk starts besides dynamic ones (Appendix A rejects
                             only BTYPE 11): GZ_START_STORED also takes stored blocks whose padding is zero,
                             LEN/NLEN complements and LEN > 1 KiB.  0: dynamic only.  Fixed blocks are not
                             offered (GZ_E_ARG): with no table to check, the fixed code resynchronises
                             inside other blocks and most candidates would be false starts */
  uint32_t reserved[2];
} gz_opts;

/* One file of a batch. */
typedef struct gz_job {
  const void *d_comp;     /* device pointer to the whole .gz file */
  uint64_t comp_len;      /* bytes */
  int32_t n_chunks;       /* 0: derived from opts.chunk_bytes */
  int32_t pad;
  void *d_out;            /* device output buffer (may be NULL at plan time for gz_decompress) */
  uint64_t out_cap;       /* bytes available at d_out */
} gz_job;

typedef struct gz_info {
  uint64_t ws_bytes;       /* workspace needed by gz_decompress* */
  uint64_t payload_start;  /* first member: byte where the DEFLATE data begins (file 0 of a batch) */
  uint64_t payload_end;    /* byte where the trailer begins (comp_len - 8) */
  uint32_t n_files;
  uint32_t n_chunks;       /* total over the batch */
  uint32_t crc32;          /* trailer CRC-32 (file 0) */
  uint32_t isize;          /* trailer ISIZE (file 0): length mod 2^32, never a size */
} gz_info;

typedef struct gz_result {
  int32_t status;          /* GZ_OK or GZ_E_* for this file */
  uint32_t n_chunks;
  uint64_t out_len;        /* decompressed bytes (valid when status is OK or CAPACITY) */
  uint64_t out_needed;     /* output bytes needed when out_cap was too small */
  uint64_t ws_needed;      /* workspace bytes a re-plan needs when a chunk overflowed (0 otherwise) */
  uint32_t n_nonempty;     /* chunks that decoded at least one block */
  uint32_t n_repairs;      /* chunks re-decoded because a start was not on the block chain */
  uint32_t n_extended;     /* chunks that continued past their first stop */
  uint32_t n_retries;      /* candidate starts rejected by the trial decode */
  uint64_t n_syms;         /* Huffman literal/length symbols decoded (end-of-block included) */
  uint64_t n_placeholders; /* symbols that referenced a chunk's unknown window */
  uint64_t n_blocks;
  uint32_t crc32;          /* CRC-32 of the output, computed on the device (when the decode succeeded) */
  uint32_t inflate_waves;  /* decoding waves of the persistent pass-1 grid (one chunk at a time each) */
} gz_result;

typedef struct gz_plan_s *gz_plan_t;

/* Plan one gzip file held at d_comp (device memory, comp_len bytes).
 * Reads the member header and the 8-byte trailer with two small synchronous
 * device-to-host copies, checks the header (RFC 1952 section 2.3), and lays
 * out the chunks: chunk i covers the compressed bytes
 * [h + floor(i*P/N), h + floor((i+1)*P/N)) of the payload (h = payload start,
 * P = payload bytes, N = n_chunks; 0 means P / opts.chunk_bytes).
 * opts may be NULL.  On success *plan owns a host object released by
 * gz_plan_destroy.  Errors: GZ_E_ARG, GZ_E_HEADER, GZ_E_HIP. */
int gz_plan(gz_plan_t *plan, const void *d_comp, size_t comp_len, int n_chunks, const gz_opts *opts);

/* Plan a batch of n_jobs files decoded together by one launch sequence. */
int gz_plan_batch(gz_plan_t *plan, const gz_job *jobs, int n_jobs, const gz_opts *opts);

int gz_plan_info(gz_plan_t plan, gz_info *info);

/* Enqueue the whole path for a one-file plan on `stream` (a hipStream_t;
 * NULL is the default stream): upload of the job table, block-start scan,
 * symbolic inflate, stitch check and repair, size scan, window propagation,
 * translation into d_out.  d_ws must hold gz_info.ws_bytes bytes and be
 * 256-byte aligned.  Returns without waiting.  Errors: GZ_E_ARG,
 * GZ_E_CAPACITY (ws_bytes too small), GZ_E_HIP. */
int gz_decompress(gz_plan_t plan, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * as gz_decompress, with the workspace taken from a static device array of
 * GZ_SCRATCH_BYTES bytes that each GPU the library runs on holds until the
 * process ends.  Allocates nothing.  The plan must belong to the current
 * device.  Every call on one GPU uses that GPU's one array, so calls that
 * overlap on one GPU race (use it from one stream at a time); each call
 * clears what it reads before writing it, so nothing carries over from the
 * last call.  Errors: GZ_E_ARG (a batch, probe or stream plan, or another
 * device), GZ_E_CAPACITY (the plan's ws_bytes above GZ_SCRATCH_BYTES),
 * GZ_E_HIP. */
#define GZ_SCRATCH_BYTES 268435456 /* 256 MiB */
int gz_decompress_static(gz_plan_t plan, void *d_out, size_t out_cap, void *stream);

/* Enqueue the path for every file of a batch plan, outputs at the jobs'
 * d_out.  One launch per pass covers all files and chunks. */
int gz_decompress_batch(gz_plan_t plan, void *d_ws, size_t ws_bytes, void *stream);

/* Enqueue the same path as gz_decompress_batch (or as the last gz_decompress
 * of a one-file plan, with its output) as one HIP graph: the first call, and
 * any call whose workspace or outputs differ from the captured ones, captures
 * the launch sequence on `stream` (which must not be NULL) and instantiates
 * it; later calls replay it.  The graph holds no memset nodes; the job table
 * is a copy from the plan's pinned buffer.  Not with opts.timing (GZ_E_ARG).
 * Errors as gz_decompress_batch. */
int gz_decompress_graph(gz_plan_t plan, void *d_ws, size_t ws_bytes, void *stream);

/* Choose opts.chunk_bytes (32 KiB .. 1 MiB) and opts.window_syms (512,
 * 1024 or 2048) for one file by timing each candidate on it (two runs each,
 * the second timed with HIP events on `stream`), and cache the choice per
 * (device, compressed-size class, compression-ratio class) for the process;
 * a cached choice returns at once.  *best: in, the other options; out, the
 * tuned options.  *ws_max (may be NULL): the workspace the most demanding
 * candidate needs.  d_ws == NULL: only *ws_max is computed.  Candidates whose
 * workspace exceeds ws_bytes are skipped.  d_out/out_cap as gz_decompress.
 * Errors: GZ_E_ARG, GZ_E_CAPACITY (no candidate fits), or the decompression
 * status when every candidate fails. */
int gz_autotune(const void *d_comp, size_t comp_len, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes,
                void *stream, gz_opts *best, uint64_t *ws_max);

/* Wait for the stream of the last gz_decompress* on this plan and read the
 * status and statistics of one file (file 0 for a one-file plan). */
int gz_result_get(gz_plan_t plan, int file, gz_result *res);

/* Per-chunk state after the stream completes (host copies, arrays of the
 * file's n_chunks entries): accepted start bit (UINT64_MAX: empty chunk),
 * the start the block-start checks of Appendix A accepted before any repair
 * (UINT64_MAX: none passed in the chunk's range; the first chunk: the
 * payload's first bit), end bit, symbol count |D_i|, output offset, status
 * (GZ_*) and flags (1 final block reached, 2 empty, 4 extended, 8 repaired:
 * the accepted start was not where the previous chunk stopped and was
 * replaced by that bit, 16 capacity overflow).  Any pointer may be NULL.
 * Used by tests to check each pass against the oracle. */
int gz_chunk_table(gz_plan_t plan, int file, uint64_t *start, uint64_t *cand, uint64_t *end, uint64_t *len,
                   uint64_t *out_off, int32_t *status, uint32_t *flags);

/* Per-chunk statistics after the stream completes (arrays of the file's
 * n_chunks entries; any pointer may be NULL):
 *   n_syms, n_placeholders, n_blocks: Huffman literal/length codes decoded
 *     (end-of-block included), symbols of D_i that are placeholders U_j, and
 *     blocks decoded, for the chunk's accepted decode (0 for an empty chunk);
 *     n_placeholders / |D_i| is the share of the chunk's output that
 *     depended on the unknown context (Section IV-C, Fig. 2);
 *   scan_cand: the smallest bit of the chunk's range that passed the static
 *     checks of the block-start search (UINT64_MAX: none);
 *   stage1, stage2: candidates that passed the cheap header checks and were
 *     given the full code-table check, and those that passed it;
 *   trial_rej, confirm_rej: candidates rejected by the trial block (ASCII
 *     literals, 1 KiB < size < 4 MiB) and by the five confirmation blocks
 *     (Appendix A).
 * The search stops at the first candidate that passes, and several
 * workgroups search one chunk at once, so the stage counts cover the bits
 * searched, not the whole range, and may differ between runs. */
int gz_chunk_stats(gz_plan_t plan, int file, uint64_t *n_syms, uint64_t *n_placeholders, uint32_t *n_blocks,
                   uint64_t *scan_cand, uint32_t *stage1, uint32_t *stage2, uint32_t *trial_rej,
                   uint32_t *confirm_rej);

/* Device addresses of a file's per-chunk symbol arrays and windows inside the
 * workspace of the last call (for tests): symbols of chunk c start at
 * sym_base + 2*sym_off[c]; its resolved window at win_base + 32768*c. */
int gz_debug_layout(gz_plan_t plan, int file, uint64_t *sym_off, uint64_t *win_index, void **sym_base,
                    void **win_base);

/* Passes timed when opts.timing is set, in launch order. */
#define GZ_N_PASSES 13
/* Names: upload, init, scan, capacity, inflate, confirm, redo, stitch,
 * finalize, tilescan, propagate, translate, crc.  Waits for the last launch and writes the duration of
 * each pass in milliseconds (HIP events on the launch stream) into ms[0..n).
 * Returns the number written, or GZ_E_NOT_READY without timing. */
int gz_pass_times(gz_plan_t plan, float *ms, int n);
const char *gz_pass_name(int i);

void gz_plan_destroy(gz_plan_t plan);
const char *gz_strerror(int code);

/* Device count and compute-unit count of device `dev` (for sizing). */
int gz_device_info(int dev, int *n_cu, int *lds_bytes);

/* ------------------------------------------------------------------------
 * Bounded-memory streaming.  Section VI-C decodes a whole member at once and
 * holds all of its output; the paper remarks (end of Section VI-C, and in the
 * Discussion) that memory could be bounded by processing one part of the
 * file at a time.  A stream
 * decodes the payload in segments of about segment_bytes compressed bytes,
 * each one run of the whole two-pass path over its own chunks:
 *   - its first chunk starts at the bit where the previous segment stopped, a
 *     block boundary reached by decoding (no block-start search), with the
 *     previous output's last 32 KiB as its context (Section IV-A's random
 *     access: a block start and a known window give the exact output);
 *   - its last chunk decodes until the first block header at or past
 *     start + 8 * segment_bytes bits (or to the member's final block).
 * Segment outputs, in order, are the member's gunzip.  The running CRC-32
 * and length are carried on, and the trailer is checked after the final
 * block.  (bit offset, window, CRC-32, length) is a checkpoint: a stream
 * resumed from it produces the same bytes as one that got there itself.
 *
 * Several members (concatenated gzip files, or BGZF-style blocked files,
 * which the paper leaves unhandled: Section VIII): a member's trailer is the
 * 8 bytes after its final block, and when more bytes follow they must be
 * the next member, which the stream then decodes from its header with a new
 * window, length and CRC-32 (RFC 1952 section 2.2).  Segment outputs, in
 * order, are then the gunzip of the whole input.
 *
 * Memory: the caller provides, per segment, an output buffer and a workspace
 * (gz_stream_get_info gives sizes that fit every segment at the options'
 * symbol factor), both valid until gz_stream_wait returns; the library
 * allocates no device memory.  The carried window goes from the segment's
 * workspace to a 32 KiB pinned host buffer of the stream (gz_stream_wait)
 * and back into the next segment's workspace.  The compressed input stays
 * caller-owned and must stay valid while the stream is used.  One stream,
 * one host thread.
 * ------------------------------------------------------------------------ */
typedef struct gz_stream_s *gz_stream_t;

typedef struct gz_stream_info {
  uint64_t ws_bytes;       /* workspace for any segment */
  uint64_t out_bytes;      /* output capacity for any segment at the symbol factor (a segment that
                              needs more reports GZ_E_CAPACITY with the size) */
  uint64_t segment_bytes;  /* compressed bytes per segment, nominal */
  uint64_t payload_start;  /* byte where the DEFLATE data begins */
  uint64_t payload_end;    /* byte where the trailer begins */
  uint32_t crc32;          /* trailer CRC-32 */
  uint32_t isize;          /* trailer ISIZE */
} gz_stream_info;

typedef struct gz_segment_result {
  int32_t status;          /* GZ_OK or GZ_E_*; after an error the stream stays where it was */
  uint32_t done;           /* 1: the input is finished (the last member's final block was decoded) */
  uint64_t out_len;        /* bytes this segment wrote at d_out */
  uint64_t out_total;      /* bytes decoded so far (all members), this segment included */
  uint64_t start_bit;      /* the segment decoded [start_bit, end_bit) of the .gz file */
  uint64_t end_bit;
  uint64_t out_needed;     /* GZ_E_CAPACITY: output bytes this segment needs */
  uint64_t ws_needed;      /* GZ_E_CAPACITY: workspace a retry needs (gz_stream_get_info has it too) */
  uint32_t crc32;          /* CRC-32 of the member's bytes so far */
  uint32_t n_chunks;
  uint32_t n_repairs;
  uint32_t n_retries;
  uint32_t member;         /* index of the member this segment decoded (0 for the first) */
  uint32_t member_done;    /* 1: the segment ended that member (its CRC-32 and ISIZE were checked) */
} gz_segment_result;

typedef struct gz_checkpoint {
  uint64_t bit;            /* where the next segment starts, in bits from the start of the .gz file */
  uint64_t out_total;      /* bytes decoded before it (all members) */
  uint64_t member_out;     /* of those, the bytes of the current member */
  uint32_t member;         /* index of the current member */
  uint32_t pad;
  uint32_t crc32;          /* CRC-32 of the current member's bytes */
  uint32_t valid;          /* real history bytes at the end of window: min(member_out, 32768) */
  uint32_t done;           /* the member is finished */
  uint32_t flags;          /* 1: a stream opened inside the member (gz_stream_open_at); valid is 32768 */
  uint8_t window[32768];   /* the 32768 bytes before `bit` (the first 32768 - valid are zero) */
} gz_checkpoint;

/* Reads the member header and trailer (small synchronous copies) and
 * allocates the pinned host window buffer.  segment_bytes 0: 256 MiB.
 * Errors: GZ_E_ARG, GZ_E_HEADER, GZ_E_HIP. */
int gz_stream_open(gz_stream_t *stream, const void *d_comp, size_t comp_len, uint64_t segment_bytes,
                   const gz_opts *opts);
int gz_stream_get_info(gz_stream_t stream, gz_stream_info *info);
/* Enqueue the next segment on hip_stream; its output goes to d_out[0 ..).
 * Then call gz_stream_wait before the next call.  Errors: GZ_E_ARG (also
 * when the member is finished or a segment is still unread),
 * GZ_E_CAPACITY (workspace too small), GZ_E_HIP. */
int gz_stream_next(gz_stream_t stream, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes,
                   void *hip_stream);
/* Wait for the segment (with the same deadline as gz_result_get) and
 * advance the stream if it succeeded.  After a capacity error the stream
 * raises its symbol factor as needed; gz_stream_get_info then gives the
 * larger sizes.  When a member ends before the input does, the next
 * member's header is read (a small synchronous copy): bytes that are not a
 * gzip member give GZ_E_HEADER (the segment's bytes are still valid). */
int gz_stream_wait(gz_stream_t stream, gz_segment_result *res);
/* Copy the position after the last finished segment (synchronous). */
int gz_stream_checkpoint(gz_stream_t stream, gz_checkpoint *cp);
/* Continue from a checkpoint of a stream over the same input.  Errors:
 * GZ_E_ARG (a bit outside the input, valid > 32768, valid differing from
 * min(member_out, 32768)), GZ_E_HIP. */
int gz_stream_resume(gz_stream_t stream, const gz_checkpoint *cp);
void gz_stream_destroy(gz_stream_t stream);

/* Concatenated gzip members (a "multi-part" file, which Section VIII lists
 * as a limitation of the paper's tool): every member is decoded by the whole
 * two-pass path, its chunks in parallel, and checked against its own
 * trailer; the outputs go back to back at d_out.  A member's end is known
 * only once its final block is decoded (a gzip header may also occur inside
 * compressed data), so the members are decoded one after another and the
 * call waits for each (synchronous, on `stream`).  d_ws == NULL: only
 * *ws_needed (the workspace for the largest possible member) is set.
 * *out_len: bytes written; *n_members: members finished.  Errors: GZ_E_ARG,
 * GZ_E_HEADER (bytes after a member that are not a member), GZ_E_CAPACITY
 * (d_out full before the input ends, or the workspace too small after a
 * raised symbol factor: *ws_needed gives the size), the first failing
 * member's status (GZ_E_DATA, GZ_E_CRC, GZ_E_SIZE), GZ_E_HIP. */
int gz_decompress_members(const void *d_comp, size_t comp_len, void *d_out, size_t out_cap, void *d_ws,
                          size_t ws_bytes, const gz_opts *opts, void *stream, uint64_t *out_len,
                          uint32_t *n_members, uint64_t *ws_needed);

/* BGZF-style input (RFC 1952 members whose extra field holds the 'BC'
 * subfield with the member's size; the paper's experiments excluded such
 * blocked files, Section VII): every member is a file of one batch plan,
 * their outputs back to back at d_out in member order, decoded in one
 * launch sequence by gz_decompress_batch (each member has its own empty
 * context, so nothing crosses members).  The member sizes, CRC-32s and
 * ISIZEs are read on the host from h_comp, a host copy of the input (NULL:
 * the library copies d_comp to the host).  *out_len: the output length (the
 * sum of the ISIZEs); *n_members: the number of files of the plan, whose
 * statuses gz_result_get gives.  d_out may be NULL to learn *out_len.
 * Errors: GZ_E_ARG, GZ_E_HEADER (a member without the subfield, or bytes
 * after the last member), GZ_E_CAPACITY (out_cap below *out_len), GZ_E_HIP. */
int gz_plan_bgzf(gz_plan_t *plan, const void *d_comp, const void *h_comp, size_t comp_len, void *d_out,
                 size_t out_cap, const gz_opts *opts, uint64_t *out_len, uint32_t *n_members);

/* ------------------------------------------------------------------------
 * Random access (Section IV).  Decoding from inside a member needs a block
 * start and the 32 KiB context before it (Section IV-A).  The start is
 * found by the block-start checks of Section VI-A and Appendix A; the
 * context is taken as undetermined (Section IV-B): 32768 copies of a marker
 * byte, which matches then copy forward exactly as they would copy the true
 * bytes, so every output byte equal to the marker is undetermined (choose a
 * marker absent from the data, e.g. 0 or 255 for text).  The share of
 * markers per window of the output is the measurement of Section IV-C and
 * Fig. 2.
 * ------------------------------------------------------------------------ */

/* Plan n_probes block-start searches in one gzip member: probe i looks for
 * the first bit b in [bits[i], bits[i] + 8 * range_bytes) (clipped to the
 * payload) that passes the static checks, the trial block and the five
 * confirmation blocks (Appendix A).  bits are counted from the start of the
 * .gz file and must lie in the payload.  range_bytes 0: 1 MiB.  The
 * workspace size is gz_plan_info's ws_bytes.  Errors: GZ_E_ARG, GZ_E_HEADER,
 * GZ_E_HIP. */
int gz_plan_probes(gz_plan_t *plan, const void *d_comp, size_t comp_len, const uint64_t *bits, int n_probes,
                   uint64_t range_bytes, const gz_opts *opts);
/* Enqueue the searches of a probe plan (one wave per probe, all at once). */
int gz_find_blocks(gz_plan_t plan, void *d_ws, size_t ws_bytes, void *stream);
/* Wait and copy each probe's block start (all-ones where none passed in
 * its range) and the candidates it rejected after the static checks. */
int gz_probe_starts(gz_plan_t plan, uint64_t *start_bits, uint32_t *n_retries);

/* A stream (see gz_stream_open) that starts at block_bit, a block start
 * inside the member (e.g. from gz_probe_starts), with the undetermined
 * context of `marker` bytes.  Its segments carry windows as any stream; the
 * trailer's CRC-32 and ISIZE are not checked (the bytes before block_bit are
 * not decoded).  Errors: as gz_stream_open, and GZ_E_ARG for a bit outside
 * the payload or a marker above 255. */
int gz_stream_open_at(gz_stream_t *stream, const void *d_comp, size_t comp_len, uint64_t block_bit, uint32_t marker,
                      uint64_t segment_bytes, const gz_opts *opts);

/* Enqueue: d_counts[(first + i) / window] += (d_buf[i] == value) for i < n,
 * windows at or past n_counts not counted (device buffers; the counts are
 * added to, so consecutive segments can share one array).  Errors: GZ_E_ARG
 * (window 0, value above 255), GZ_E_HIP. */
int gz_count_byte(const void *d_buf, uint64_t n, uint32_t value, uint64_t first, uint64_t window, uint64_t *d_counts,
                  uint64_t n_counts, void *stream);

/* DNA-like sequences in partly undetermined text (Appendix B), and the
 * sequence-resolved test of Section VI-B.  Scanning left to right, every
 * maximal substring T D+ (U+ D+)* T is taken, where D is a nucleotide letter
 * (upper-case A, C, G, T or N), U an undetermined element and T a newline
 * or an undetermined element; the earliest start wins, then the longest
 * match from it, and the search resumes after the closing T (so a newline
 * that closes one sequence does not open the next).  A sequence is the
 * match without its two T's; sequences shorter than min_len are dropped
 * after the search.
 *   d_buf, n      the text: elem_bytes 1, bytes in which the value `marker`
 *                 is undetermined (the output of a random-access stream,
 *                 Section IV-B); elem_bytes 2, 16-bit symbols in which every
 *                 value of 256 and above is undetermined (pass-1 symbols,
 *                 Section VI-C; marker ignored).  n below 2^32.
 *   d_seqs        the first max_seqs sequences, in order (may be NULL when
 *                 max_seqs is 0); *d_n_seqs receives the total found.
 *   d_bounds      n_ranges + 1 ascending positions (e.g. the output offsets of
 *                 DEFLATE blocks); a sequence counts in the range holding its
 *                 first nucleotide.  d_range_stats gets 3 words per range:
 *                 sequences, sequences holding an undetermined element, and
 *                 1 when the first is at least `threshold` and the second 0
 *                 (the range is sequence-resolved).  n_ranges 0: no ranges.
 *   d_ws          gz_extract_dna_ws(n) bytes, 256-byte aligned.
 * Every buffer is device memory owned by the caller; the call only enqueues
 * on `stream`.  Errors: GZ_E_ARG (elem_bytes not 1 or 2, n too large, a
 * marker above 255 or equal to a nucleotide letter or newline, a missing
 * buffer), GZ_E_CAPACITY (ws_bytes too small), GZ_E_HIP. */
typedef struct gz_dna_seq {
  uint64_t start;           /* position of the first nucleotide */
  uint32_t len;             /* elements in the sequence */
  uint32_t n_undetermined;  /* undetermined elements inside it */
} gz_dna_seq;

uint64_t gz_extract_dna_ws(uint64_t n);
int gz_extract_dna(const void *d_buf, uint64_t n, uint32_t elem_bytes, uint32_t marker, uint32_t min_len,
                   gz_dna_seq *d_seqs, uint64_t max_seqs, uint64_t *d_n_seqs, const uint64_t *d_bounds,
                   uint32_t n_ranges, uint32_t threshold, uint32_t *d_range_stats, void *d_ws, size_t ws_bytes,
                   void *stream);

/* ------------------------------------------------------------------------
 * Serving loop (beyond the paper's one-file setting): jobs arrive one at a
 * time and are admitted into batches while two bounds hold: the footprints
 * of the jobs in flight (compressed input + output capacity + workspace)
 * stay within the HBM budget, and the batch's workspace fits in the
 * caller's device arena.  Batches run as batched launch sequences on up to
 * max_inflight streams at once; a finished batch frees its arena block and
 * its share of the budget for the jobs queued behind it (continuous
 * batching).  The library allocates no device memory: the arena, the inputs
 * and the outputs are the caller's, and must stay valid until the server is
 * destroyed (the arena) or the job is reported done (its buffers).
 * Single-threaded: every call on one server comes from one host thread.
 * ------------------------------------------------------------------------ */
typedef struct gz_server_s *gz_server_t;

typedef struct gz_server_opts {
  void *arena;            /* device memory for the batches' workspaces, owned by the caller, 256-byte aligned */
  uint64_t arena_bytes;   /* bytes at arena (at least 4096) */
  uint64_t budget_bytes;  /* HBM budget of the jobs in flight: inputs + outputs + workspaces (0: arena_bytes) */
  uint32_t max_inflight;  /* batches in flight, one non-blocking stream each (default 4) */
  uint32_t max_batch;     /* jobs per batch (default 64) */
  gz_opts opts;           /* decompression options of every job */
} gz_server_opts;

typedef struct gz_done {
  uint64_t tag;           /* as given to gz_server_submit */
  int32_t status;         /* GZ_OK or a GZ_E_* code (GZ_E_CAPACITY: output too small, or larger than the
                             arena or the budget) */
  uint32_t pad;
  uint64_t out_len;       /* decompressed bytes written at d_out */
  double t_submit;        /* seconds since the server was created: submission, */
  double t_start;         /* launch of its batch, */
  double t_end;           /* and the poll that saw the batch finished */
} gz_done;

typedef struct gz_server_info {
  uint32_t queued, running, finished_unread;
  uint32_t mem_waited;    /* jobs whose admission waited for the budget or the arena (at least once) */
  uint64_t batches;       /* batches launched so far */
  uint64_t arena_bytes, arena_used, arena_peak;  /* workspaces in the arena */
  uint64_t budget_bytes, resident, resident_peak; /* footprints of the jobs in flight */
  double now;             /* seconds since creation */
} gz_server_info;

/* Errors: GZ_E_ARG (no arena, or one not 256-byte aligned), GZ_E_HIP (the
 * streams could not be made). */
int gz_server_create(gz_server_t *server, const gz_server_opts *opts);
/* Queue one job (plans it alone to estimate its workspace: reads its gzip
 * header and trailer).  Errors: GZ_E_ARG, GZ_E_HEADER, GZ_E_HIP. */
int gz_server_submit(gz_server_t server, const void *d_comp, size_t comp_len, void *d_out, size_t out_cap,
                     uint64_t tag);
/* Reap finished batches (a job that ran out of symbol capacity is queued
 * again, first, with 4x the capacity factor), admit queued jobs in order
 * while a stream is free and their workspaces fit, and copy up to max_done
 * finished jobs to done[].  Never waits for the GPU.  Returns the number
 * copied, or a GZ_E_* code when a launch failed. */
int gz_server_poll(gz_server_t server, gz_done *done, int max_done);
int gz_server_stats(gz_server_t server, gz_server_info *info);
/* Waits for the batches in flight, then frees everything. */
void gz_server_destroy(gz_server_t server);

#ifdef __cplusplus
}
#endif
#endif
