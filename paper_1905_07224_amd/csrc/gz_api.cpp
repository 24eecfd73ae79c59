// C ABI of the two-pass gzip path: planning on the host, launch sequence on a
// HIP stream, result read-back.  See include/gzgpu.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/gzgpu.h"
#include "gz_internal.h"

using namespace gzgpu;

extern "C" {
hipError_t gzk_init(ChunkState *, uint32_t, FileState *, uint32_t, Counters *, hipStream_t);
hipError_t gzk_scan(const FileDesc *, const ChunkDesc *, ChunkState *, const uint32_t *, uint32_t, uint32_t,
                    hipStream_t);
hipError_t gzk_capacity(uint32_t, const FileDesc *, ChunkDesc *, const ChunkState *, uint32_t, hipStream_t);
hipError_t gzk_inflate(int, uint32_t, uint32_t, const FileDesc *, const ChunkDesc *, ChunkState *, const uint32_t *,
                       uint32_t, Counters *, uint16_t *, hipStream_t);
hipError_t gzk_confirm(int, uint32_t, const FileDesc *, const ChunkDesc *, ChunkState *, uint32_t, Counters *,
                       uint16_t *, uint32_t, hipStream_t);
hipError_t gzk_redo(int, uint32_t, const FileDesc *, const ChunkDesc *, ChunkState *, uint32_t, Counters *, uint16_t *,
                    hipStream_t);
hipError_t gzk_stitch(int, uint32_t, const FileDesc *, const ChunkDesc *, ChunkState *, uint32_t, Counters *,
                      uint16_t *, hipStream_t);
hipError_t gzk_finalize(int, uint32_t, const FileDesc *, const ChunkDesc *, ChunkState *, FileState *, uint16_t *,
                        hipStream_t);
hipError_t gzk_crc(uint32_t, const FileDesc *, FileState *, const uint32_t *, uint64_t, hipStream_t);
hipError_t gzk_tilescan(const ChunkDesc *, const ChunkState *, const FileState *, uint32_t, uint64_t *, uint32_t *,
                        AccEntry *, hipStream_t);
hipError_t gzk_propagate(uint32_t, const uint32_t *, const AccEntry *, uint8_t *, const uint16_t *, uint16_t *,
                         uint8_t *, hipStream_t);
hipError_t gzk_translate(uint32_t, const FileDesc *, const ChunkDesc *, const ChunkState *, FileState *,
                         const uint64_t *, uint32_t, const uint8_t *, const uint16_t *, Counters *, hipStream_t);
hipError_t gzk_carry(const FileDesc *, const FileState *, const uint8_t *, uint8_t *, hipStream_t);
hipError_t gzk_scratch(void **);
hipError_t gzk_count_byte(const uint8_t *, uint64_t, uint32_t, uint64_t, uint64_t, unsigned long long *, uint64_t,
                          hipStream_t);
uint64_t gzk_dna_ws(uint64_t);
hipError_t gzk_dna(const void *, uint64_t, uint32_t, uint32_t, uint32_t, gz_dna_seq *, uint64_t, uint64_t *,
                   const uint64_t *, uint32_t, uint32_t, uint32_t *, uint8_t *, hipStream_t);
}

namespace {

thread_local char g_err[256];

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// CRC-32 (RFC 1952 section 8), table driven; used only for the FHCRC field.
uint32_t crc32_host(const uint8_t *p, size_t n) {
  static uint32_t tab[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; i++) {
      uint32_t c = i;
      for (int k = 0; k < 8; k++) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
      tab[i] = c;
    }
    init = true;
  }
  uint32_t c = 0xFFFFFFFFu;
  for (size_t i = 0; i < n; i++) c = tab[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
  return c ^ 0xFFFFFFFFu;
}

// gzip member header (RFC 1952 section 2.3): returns the payload start or -1.
int64_t parse_gzip_header(const uint8_t *h, size_t n) {
  if (n < 10) return -1;
  if (h[0] != 0x1f || h[1] != 0x8b || h[2] != 8) return -1;
  const unsigned flg = h[3];
  if (flg & 0xE0u) return -1;
  size_t p = 10;
  if (flg & 4u) {
    if (p + 2 > n) return -1;
    p += 2 + ((size_t)h[p] | ((size_t)h[p + 1] << 8));
    if (p > n) return -1;
  }
  for (unsigned bit : {8u, 16u}) {
    if (flg & bit) {
      while (p < n && h[p]) p++;
      if (p >= n) return -1;
      p++;
    }
  }
  if (flg & 2u) {
    if (p + 2 > n) return -1;
    const uint32_t want = (uint32_t)h[p] | ((uint32_t)h[p + 1] << 8);
    if ((crc32_host(h, p) & 0xFFFFu) != want) return -1;
    p += 2;
  }
  return (int64_t)p;
}

// x^(8 * 2^k) mod P for the device CRC combine (reflected representation:
// bit 31 is x^0; multiplying by x is a right shift that folds bit 0 back
// through the polynomial 0xEDB88320)
uint32_t gf_mulx_host(uint32_t a) { return (a >> 1) ^ (0xEDB88320u & (0u - (a & 1u))); }
uint32_t gf_mul_host(uint32_t a, uint32_t b) {
  uint32_t p = 0;
  for (int i = 0; i < 32; i++) {
    if ((a >> (31 - i)) & 1u) p ^= b;
    b = gf_mulx_host(b);
  }
  return p;
}
void crc_xpow_table(uint32_t *t) {
  uint32_t x = 0x80000000u;
  for (int i = 0; i < 8; i++) x = gf_mulx_host(x);
  t[0] = x;
  for (int k = 1; k < CRC_XPOW; k++) t[k] = gf_mul_host(t[k - 1], t[k - 1]);
  // x^(8 * CRC_LANE * m): CRC_LANE is a power of two
  int lg = 0;
  while ((1u << lg) < CRC_LANE) lg++;
  uint32_t step = t[lg], acc = 0x80000000u;
  for (int m = 0; m < 64; m++) {
    t[CRC_XPOW + m] = acc;
    acc = gf_mul_host(acc, step);
  }
}

int hip_fail(hipError_t e, const char *what) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
  return GZ_E_HIP;
}

// Device-to-host copy ordered on `st` only: the host waits for that stream,
// not for work that other streams have in flight (a plain hipMemcpy may wait
// for the whole device, which would stall a serving loop on the batches it
// is running).
hipError_t copy_to_host(void *dst, const void *src, size_t n, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

// A non-blocking stream per device for the small reads made while planning
// (gzip headers and trailers).
std::mutex g_ctl_mu;
hipStream_t g_ctl[64] = {};
hipError_t control_stream(hipStream_t *st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_ctl_mu);
  if (!g_ctl[dev]) {
    e = hipStreamCreateWithFlags(&g_ctl[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *st = g_ctl[dev];
  return hipSuccess;
}

// The autotuner's choices, per (device, compressed-size class, ratio class):
// the size class is the bit length of the compressed size, the ratio class
// four times the compression ratio (ISIZE over payload bytes), at most 64.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, gz_opts> g_tune;

std::tuple<int, int, int> tune_key(int dev, uint64_t comp_len, uint64_t payload, uint32_t isize) {
  int size_class = 0;
  while ((comp_len >> size_class) > 1) size_class++;
  const int ratio_class = (int)std::min<double>(64.0, 4.0 * (double)isize / (double)std::max<uint64_t>(1, payload));
  return std::make_tuple(dev, size_class, ratio_class);
}

bool tune_lookup(int dev, uint64_t comp_len, uint64_t payload, uint32_t isize, gz_opts *o) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_key(dev, comp_len, payload, isize));
  if (it == g_tune.end()) return false;
  *o = it->second;
  return true;
}

}  // namespace

struct gz_plan_s {
  gz_opts opts{};
  uint32_t win = 32768;
  uint32_t groups = 8;
  int n_cu = 256;
  int device = 0;
  std::vector<FileDesc> files;
  std::vector<ChunkDesc> chunks;
  std::vector<uint32_t> order;
  std::vector<uint32_t> scan_list;
  Layout lay{};
  uint64_t order_bytes = 0, scan_off = 0;
  uint8_t *pinned = nullptr;
  uint64_t pinned_bytes = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  hipEvent_t pass_ev[GZ_N_PASSES + 1] = {};
  bool timed = false;
  // captured launch sequence (gz_decompress_graph)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint8_t *graph_ws = nullptr;
  std::vector<std::pair<uint8_t *, uint64_t>> graph_out;
  bool capturing = false;
  // last launch
  uint8_t *ws = nullptr;
  hipStream_t stream = nullptr;
  bool launched = false;
  bool fetched = false;         // the stream finished and fst holds the file states
  bool fetched_chunks = false;  // cst and cdev hold the chunk states and table too
  std::vector<FileState> fst;
  std::vector<ChunkState> cst;
  std::vector<ChunkDesc> cdev;  // the device's chunk table after the run (capacities)
  std::vector<gz_job> jobs;
  std::vector<uint64_t> span;   // per file: compressed bytes its pool was sized for
  // a segment of a longer member (gz_stream_*): one file, decoded from
  // start_bit (a block boundary) to the first block at or past stop_bit
  // (NONE: to the final block), its first chunk with a carried window
  struct Segment {
    bool on = false;
    uint64_t start_bit = 0, stop_bit = NONE, out_before = 0;
    uint32_t crc_in = 0, win_valid = 0;
    uint32_t mode = 0;    // FD_NOCHECK: the stream began inside the member
    int64_t h = 0;        // payload start byte
    uint32_t crc = 0, isize = 0;
  } seg;
  // members whose header and trailer were read by the caller (gz_plan_bgzf):
  // payload start (from the member's start), trailer CRC-32 and ISIZE
  struct Member {
    int64_t h;
    uint32_t crc, isize;
  };
  std::vector<Member> pre;
  // block-start probes (gz_plan_probes): file f searches [lo, hi) of the one input
  bool probe = false;
  std::vector<uint64_t> probe_lo, probe_hi;
  bool dry = false;  // sizes only: no pinned job table (the serving loop's estimates)
};

// Header and trailer of the member at j.d_comp: payload start, CRC-32, ISIZE.
static int read_member(const gz_job &j, uint32_t f, int64_t *h_out, uint32_t *crc, uint32_t *isize) {
  if (!j.d_comp || j.comp_len < 18) {
    snprintf(g_err, sizeof(g_err), "file %u: input too short for a gzip member", f);
    return j.d_comp ? GZ_E_HEADER : GZ_E_ARG;
  }
  // header bytes (grown if the optional fields are long) and the trailer
  hipStream_t ctl = nullptr;
  hipError_t ce = control_stream(&ctl);
  if (ce != hipSuccess) return hip_fail(ce, "control stream");
  size_t hn = (size_t)std::min<uint64_t>(j.comp_len, 4096);
  std::vector<uint8_t> hb;
  int64_t h = -1;
  for (;;) {
    hb.resize(hn);
    hipError_t e = copy_to_host(hb.data(), j.d_comp, hn, ctl);
    if (e != hipSuccess) return hip_fail(e, "reading the gzip header");
    h = parse_gzip_header(hb.data(), hn);
    if (h >= 0 || hn == j.comp_len) break;
    hn = (size_t)std::min<uint64_t>(j.comp_len, (uint64_t)hn * 4);
  }
  if (h < 0 || (uint64_t)h + 8 >= j.comp_len) {
    snprintf(g_err, sizeof(g_err), "file %u: invalid gzip member header", f);
    return GZ_E_HEADER;
  }
  uint8_t tr[8];
  hipError_t e = copy_to_host(tr, (const uint8_t *)j.d_comp + j.comp_len - 8, 8, ctl);
  if (e != hipSuccess) return hip_fail(e, "reading the gzip trailer");
  *h_out = h;
  *crc = (uint32_t)tr[0] | ((uint32_t)tr[1] << 8) | ((uint32_t)tr[2] << 16) | ((uint32_t)tr[3] << 24);
  *isize = (uint32_t)tr[4] | ((uint32_t)tr[5] << 8) | ((uint32_t)tr[6] << 16) | ((uint32_t)tr[7] << 24);
  return GZ_OK;
}

// Chunks the persistent inflate grid decodes at once (one wave each).
static uint64_t decode_slots(gz_plan_t p) {
  const uint32_t lds_per_cu = 160 * 1024;
  const uint32_t per_wave = inflate_lds_bytes(p->win) + 256;
  const uint32_t waves_per_cu = p->opts.inflate_waves_per_cu ? p->opts.inflate_waves_per_cu
                                                             : std::max<uint32_t>(1, lds_per_cu / per_wave);
  return (uint64_t)waves_per_cu * (uint64_t)std::max(1, p->n_cu);
}

static bool valid_ring(uint32_t win);

static int plan_common(gz_plan_t p) {
  const uint32_t F = (uint32_t)p->jobs.size();
  uint64_t tuned_len = 0;
  uint32_t tuned_win = 0;
  p->files.clear();
  p->chunks.clear();
  p->span.clear();
  uint64_t sym_elems = 0;
  for (uint32_t f = 0; f < F; f++) {
    const gz_job &j = p->jobs[f];
    int64_t h = 0;
    uint32_t crc = 0, isize = 0;
    if (!p->pre.empty()) {
      h = p->pre[f].h;
      crc = p->pre[f].crc;
      isize = p->pre[f].isize;
    } else if (p->seg.on || (p->probe && f > 0)) {
      h = p->seg.h;
      crc = p->seg.crc;
      isize = p->seg.isize;
    } else {
      const int r = read_member(j, f, &h, &crc, &isize);
      if (r != GZ_OK) return r;
      p->seg.h = h;
      p->seg.crc = crc;
      p->seg.isize = isize;
    }
    FileDesc fd{};
    fd.comp = (const uint8_t *)j.d_comp;
    fd.comp_len = j.comp_len;
    fd.payload_bit = 8ull * (uint64_t)h;
    fd.trailer_byte = j.comp_len - 8;
    fd.out = (uint8_t *)j.d_out;
    fd.out_cap = j.out_cap;
    fd.crc = crc;
    fd.isize = isize;
    fd.stop_bit = NONE;
    // chunks cut the bytes [lo, hi): the payload, or a segment's range
    uint64_t lo = (uint64_t)h, hi = fd.trailer_byte, margin = 0;
    if (p->probe) {
      // one chunk searching [probe_lo, probe_hi) bits; it decodes one block
      // and its confirmation
      fd.mode = FD_PROBE | (p->opts.binary ? FD_BINARY : 0u) |
                ((p->opts.start_types & GZ_START_STORED) ? FD_STORED_STARTS : 0u);
      fd.stop_bit = p->probe_hi[f];
      fd.first_chunk = (uint32_t)p->chunks.size();
      fd.n_chunks = 1;
      ChunkDesc cd{};
      cd.lo_bit = p->probe_lo[f];
      cd.hi_bit = p->probe_hi[f];
      cd.file = f;
      p->chunks.push_back(cd);
      fd.pool_base = sym_elems;
      fd.pool_elems = (uint64_t)p->opts.sym_factor * (STOP_MARGIN_BYTES + 1) + SYM_SLACK + FLUSH_UNIT;
      sym_elems += align_up(fd.pool_elems, FLUSH_UNIT);
      p->span.push_back(STOP_MARGIN_BYTES + 1);
      p->files.push_back(fd);
      continue;
    }
    if (p->seg.on) {
      fd.payload_bit = p->seg.start_bit;
      lo = (p->seg.start_bit + 7) / 8;
      if (p->seg.stop_bit != NONE && p->seg.stop_bit < 8 * fd.trailer_byte) {
        fd.stop_bit = p->seg.stop_bit;
        hi = std::max<uint64_t>(lo + 1, p->seg.stop_bit / 8);
        margin = STOP_MARGIN_BYTES;
      }
      fd.out_before = p->seg.out_before;
      fd.crc_in = p->seg.crc_in;
      fd.win_valid = p->seg.win_valid;
      fd.mode = p->seg.mode;
    }
    if (p->opts.binary) fd.mode |= FD_BINARY;
    if (p->opts.start_types & GZ_START_STORED) fd.mode |= FD_STORED_STARTS;
    const uint64_t P = hi > lo ? hi - lo : 1;
    uint64_t cb = p->opts.chunk_bytes;
    if (p->opts.tuned && !p->seg.on) {
      // the autotuner's chunk size for this file's class, when it has one;
      // the ring of the largest such file
      gz_opts t;
      if (tune_lookup(p->device, j.comp_len, P, isize, &t) && t.chunk_bytes) {
        cb = t.chunk_bytes;
        if (!p->opts.window_syms && j.comp_len >= tuned_len && valid_ring(t.window_syms)) {
          tuned_len = j.comp_len;
          tuned_win = t.window_syms;
        }
      }
    }
    uint64_t N = j.n_chunks > 0 ? (uint64_t)j.n_chunks : (P + cb - 1) / cb;
    N *= std::max<uint32_t>(1, p->opts.waves_per_chunk);
    N = std::max<uint64_t>(1, std::min<uint64_t>(N, P));
    fd.first_chunk = (uint32_t)p->chunks.size();
    fd.n_chunks = (uint32_t)N;
    for (uint64_t i = 0; i < N; i++) {
      ChunkDesc cd{};
      const uint64_t a = lo + (uint64_t)((unsigned __int128)i * P / N);
      const uint64_t b = lo + (uint64_t)((unsigned __int128)(i + 1) * P / N);
      cd.lo_bit = i == 0 ? fd.payload_bit : 8 * a;
      cd.hi_bit = 8 * b;
      cd.file = f;
      cd.index = (uint32_t)i;
      cd.flags = i == 0 ? (CF_FIRST | (p->seg.on && p->seg.win_valid ? CF_CARRIED : 0u)) : 0u;
      p->chunks.push_back(cd);
    }
    // the chunks' capacities are set on the device from their actual spans;
    // their sum is bounded by this
    fd.pool_base = sym_elems;
    // spans to the next candidate (partitioning the payload) plus, at most,
    // half of every chunk's range (see k_capacity)
    const uint64_t span_sum = P + margin + N + (P + N) / 2 + N;
    fd.pool_elems = (uint64_t)p->opts.sym_factor * span_sum + N * (SYM_SLACK + FLUSH_UNIT);
    p->span.push_back(span_sum);
    sym_elems += align_up(fd.pool_elems, FLUSH_UNIT);
    p->files.push_back(fd);
  }
  if (tuned_win) p->win = tuned_win;
  const uint32_t N = (uint32_t)p->chunks.size();
  // workgroups per chunk search: enough for some 4096 in all
  if (!p->opts.scan_groups) p->groups = std::max<uint32_t>(1, std::min<uint32_t>(64, 4096 / std::max<uint32_t>(1, N)));
  // inflate order: longest compressed range first
  p->order.resize(N);
  for (uint32_t i = 0; i < N; i++) p->order[i] = i;
  std::stable_sort(p->order.begin(), p->order.end(), [&](uint32_t x, uint32_t y) {
    return (p->chunks[x].hi_bit - p->chunks[x].lo_bit) > (p->chunks[y].hi_bit - p->chunks[y].lo_bit);
  });
  p->scan_list.clear();
  for (uint32_t i = 0; i < N; i++)
    if (!(p->chunks[i].flags & CF_FIRST)) p->scan_list.push_back(i);
  // workspace layout
  Layout &L = p->lay;
  uint64_t o = 0;
  L.files_off = o;
  o = align_up(o + F * sizeof(FileDesc), 256);
  L.chunks_off = o;
  o = align_up(o + (uint64_t)N * sizeof(ChunkDesc), 256);
  L.order_off = o;
  o = align_up(o + (uint64_t)N * 4, 256);
  p->scan_off = o;
  o = align_up(o + (uint64_t)p->scan_list.size() * 4 + 4, 256);
  L.crc_off = o;
  o = align_up(o + CRC_CONSTS * 4, 256);
  L.table_bytes = o;
  L.cstate_off = o;
  o = align_up(o + (uint64_t)N * sizeof(ChunkState), 256);
  L.fstate_off = o;
  o = align_up(o + F * sizeof(FileState), 256);
  L.counters_off = o;
  o = align_up(o + sizeof(Counters), 256);
  L.tiles_off = o;
  o = align_up(o + ((uint64_t)N + 1) * 8, 256);
  L.acc_off = o;
  o = align_up(o + ((uint64_t)N + 1) * 4, 256);
  o = align_up(o + (uint64_t)N * sizeof(AccEntry), 256);
  const uint64_t nseg = (N + 63) / 64;
  L.maps_off = o;  // two map arrays: the prefix composition alternates between them
  o = align_up(o + 2 * nseg * WINDOW * 2, 256);
  L.segwin_off = o;
  o = align_up(o + nseg * WINDOW, 256);
  L.win_off = o;
  o = align_up(o + (uint64_t)N * WINDOW, 256);
  L.carry_off = o;
  o = align_up(o + (p->seg.on ? WINDOW : 0), 256);
  L.sym_off = o;
  L.sym_elems = sym_elems;
  o = align_up(o + sym_elems * 2, 256);
  L.total = o;
  // pinned copy of the job table (kept when a re-plan fits in it; the last
  // upload from it has finished before it is rewritten, see launch)
  if (p->dry) return GZ_OK;
  if (p->pinned && p->pinned_bytes >= L.table_bytes) return GZ_OK;
  if (p->pinned) {
    if (p->upload_pending) {
      (void)hipEventSynchronize(p->upload_done);
      p->upload_pending = false;
    }
    (void)hipHostFree(p->pinned);
  }
  p->pinned = nullptr;
  p->pinned_bytes = 0;
  hipError_t e = hipHostMalloc((void **)&p->pinned, L.table_bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "pinned job table");
  p->pinned_bytes = L.table_bytes;
  return GZ_OK;
}

// Ring sizes the decoder is built for: powers of two from 512 to 32768.
static bool valid_ring(uint32_t win) { return win >= 512 && win <= 32768 && (win & (win - 1)) == 0; }

// Options a plan can run with: a ring the decoder is built for, start types it offers.
static bool valid_opts(const gz_plan_s *p) { return valid_ring(p->win) && (p->opts.start_types & ~GZ_START_STORED) == 0; }

static void fill_defaults(gz_plan_t p, const gz_opts *opts, bool query_device = true) {
  if (opts) p->opts = *opts;
  if (p->opts.chunk_bytes == 0) p->opts.chunk_bytes = DEFAULT_CHUNK_BYTES;
  if (p->opts.sym_factor == 0) p->opts.sym_factor = 8;
  // LDS history ring of each decoding wave: older match sources are read back
  // from HBM, so a smaller ring trades those reads for more waves per CU
  p->win = p->opts.window_syms ? p->opts.window_syms : DEFAULT_RING;
  p->groups = p->opts.scan_groups;
  if (!query_device) return;
  (void)hipGetDevice(&p->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) p->n_cu = prop.multiProcessorCount;
}

static int make_plan(gz_plan_t *plan, const gz_job *jobs, int n, const gz_opts *opts) {
  if (!plan || !jobs || n <= 0) return GZ_E_ARG;
  *plan = nullptr;
  gz_plan_t p = new (std::nothrow) gz_plan_s();
  if (!p) return GZ_E_ARG;
  fill_defaults(p, opts);
  if (!valid_opts(p)) {
    gz_plan_destroy(p);
    return GZ_E_ARG;
  }
  p->jobs.assign(jobs, jobs + n);
  int r = plan_common(p);
  if (r != GZ_OK) {
    gz_plan_destroy(p);
    return r;
  }
  (void)hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
  if (p->opts.timing)
    for (int i = 0; i <= GZ_N_PASSES; i++) (void)hipEventCreate(&p->pass_ev[i]);
  *plan = p;
  return GZ_OK;
}

static void drop_graph(gz_plan_t p);

extern "C" {

// Internal to the library (the serving loop): the workspace a batch of jobs
// needs, without creating a plan object (no pinned memory).
int gzi_plan_ws(const gz_job *jobs, int n, const gz_opts *opts, uint64_t *ws_bytes) {
  if (!jobs || n <= 0 || !ws_bytes) return GZ_E_ARG;
  gz_plan_s p;
  p.dry = true;
  fill_defaults(&p, opts);
  if (!valid_opts(&p)) return GZ_E_ARG;
  p.jobs.assign(jobs, jobs + n);
  const int r = plan_common(&p);
  if (r == GZ_OK) *ws_bytes = p.lay.total;
  return r;
}

// Internal to the library (the serving loop): plan a batch into an existing
// plan object whose last launch has finished, keeping its pinned job table
// and events (allocating and freeing pinned memory may wait for the device).
// *plan NULL: a new plan.
int gzi_replan(gz_plan_t *plan, const gz_job *jobs, int n, const gz_opts *opts) {
  if (!plan || !jobs || n <= 0) return GZ_E_ARG;
  if (!*plan) return make_plan(plan, jobs, n, opts);
  gz_plan_t p = *plan;
  if (p->upload_pending) {
    (void)hipEventSynchronize(p->upload_done);
    p->upload_pending = false;
  }
  drop_graph(p);
  p->launched = p->fetched = p->fetched_chunks = false;
  p->timed = false;
  const bool timing_events = p->opts.timing != 0;
  fill_defaults(p, opts, false);
  p->opts.timing = timing_events ? p->opts.timing : 0;
  if (!valid_opts(p)) return GZ_E_ARG;
  p->jobs.assign(jobs, jobs + n);
  return plan_common(p);
}

int gz_plan(gz_plan_t *plan, const void *d_comp, size_t comp_len, int n_chunks, const gz_opts *opts) {
  if (!d_comp || comp_len == 0 || n_chunks < 0) return GZ_E_ARG;
  gz_job j{};
  j.d_comp = d_comp;
  j.comp_len = comp_len;
  j.n_chunks = n_chunks;
  return make_plan(plan, &j, 1, opts);
}

int gz_plan_batch(gz_plan_t *plan, const gz_job *jobs, int n_jobs, const gz_opts *opts) {
  return make_plan(plan, jobs, n_jobs, opts);
}

static int launch(gz_plan_t p, uint8_t *ws, size_t ws_bytes, hipStream_t st);
static int fetch(gz_plan_t p);
static int fetch_chunks(gz_plan_t p);

int gz_plan_probes(gz_plan_t *plan, const void *d_comp, size_t comp_len, const uint64_t *bits, int n_probes,
                   uint64_t range_bytes, const gz_opts *opts) {
  if (!plan || !d_comp || comp_len == 0 || !bits || n_probes <= 0) return GZ_E_ARG;
  *plan = nullptr;
  gz_job j{};
  j.d_comp = d_comp;
  j.comp_len = comp_len;
  int64_t h = 0;
  uint32_t crc = 0, isize = 0;
  int r = read_member(j, 0, &h, &crc, &isize);
  if (r != GZ_OK) return r;
  const uint64_t lo_ok = 8ull * (uint64_t)h, hi_ok = 8ull * (comp_len - 8);
  const uint64_t range = range_bytes ? range_bytes : (1ull << 20);
  gz_plan_t p = new (std::nothrow) gz_plan_s();
  if (!p) return GZ_E_ARG;
  fill_defaults(p, opts);
  if (!valid_opts(p)) {
    gz_plan_destroy(p);
    return GZ_E_ARG;
  }
  p->probe = true;
  p->seg.h = h;
  p->seg.crc = crc;
  p->seg.isize = isize;
  for (int i = 0; i < n_probes; i++) {
    if (bits[i] < lo_ok || bits[i] >= hi_ok) {
      snprintf(g_err, sizeof(g_err), "probe %d: bit %llu is outside the payload", i, (unsigned long long)bits[i]);
      gz_plan_destroy(p);
      return GZ_E_ARG;
    }
    p->probe_lo.push_back(bits[i]);
    p->probe_hi.push_back(std::min<uint64_t>(hi_ok, bits[i] + 8 * range));
  }
  p->jobs.assign((size_t)n_probes, j);
  r = plan_common(p);
  if (r != GZ_OK) {
    gz_plan_destroy(p);
    return r;
  }
  (void)hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
  *plan = p;
  return GZ_OK;
}

int gz_plan_bgzf(gz_plan_t *plan, const void *d_comp, const void *h_comp, size_t comp_len, void *d_out,
                 size_t out_cap, const gz_opts *opts, uint64_t *out_len, uint32_t *n_members) {
  if (!plan || !d_comp || comp_len == 0) return GZ_E_ARG;
  *plan = nullptr;
  std::vector<uint8_t> copy;
  const uint8_t *hb = (const uint8_t *)h_comp;
  if (!hb) {
    copy.resize(comp_len);
    hipStream_t ctl = nullptr;
    hipError_t e = control_stream(&ctl);
    if (e == hipSuccess) e = copy_to_host(copy.data(), d_comp, comp_len, ctl);
    if (e != hipSuccess) return hip_fail(e, "reading the input");
    hb = copy.data();
  }
  std::vector<gz_job> jobs;
  std::vector<gz_plan_s::Member> pre;
  uint64_t at = 0, total = 0;
  while (at < comp_len) {
    const uint8_t *m = hb + at;
    const size_t left = comp_len - at;
    // the member's size from its 'BC' extra subfield (RFC 1952 section 2.3.1.1)
    uint64_t size = 0;
    if (left >= 18 && m[0] == 0x1f && m[1] == 0x8b && m[2] == 8 && (m[3] & 4u)) {
      const size_t xlen = (size_t)m[10] | ((size_t)m[11] << 8);
      for (size_t q = 12; q + 4 <= 12 + xlen && q + 4 <= left;) {
        const size_t slen = (size_t)m[q + 2] | ((size_t)m[q + 3] << 8);
        if (m[q] == 'B' && m[q + 1] == 'C' && slen == 2 && q + 6 <= left) size = ((uint64_t)m[q + 4] | ((uint64_t)m[q + 5] << 8)) + 1;
        q += 4 + slen;
      }
    }
    const int64_t h = size ? parse_gzip_header(m, (size_t)std::min<uint64_t>(size, left)) : -1;
    if (!size || size > left || h < 0 || (uint64_t)h + 8 > size) {
      snprintf(g_err, sizeof(g_err), "member at byte %llu: not a BGZF member", (unsigned long long)at);
      return GZ_E_HEADER;
    }
    const uint8_t *tr = m + size - 8;
    gz_plan_s::Member mb;
    mb.h = h;
    mb.crc = (uint32_t)tr[0] | ((uint32_t)tr[1] << 8) | ((uint32_t)tr[2] << 16) | ((uint32_t)tr[3] << 24);
    mb.isize = (uint32_t)tr[4] | ((uint32_t)tr[5] << 8) | ((uint32_t)tr[6] << 16) | ((uint32_t)tr[7] << 24);
    gz_job j{};
    j.d_comp = (const uint8_t *)d_comp + at;
    j.comp_len = size;
    j.d_out = d_out ? (uint8_t *)d_out + total : nullptr;
    j.out_cap = mb.isize;  // a BGZF member holds at most 64 KiB, so ISIZE is its length
    jobs.push_back(j);
    pre.push_back(mb);
    total += mb.isize;
    at += size;
  }
  if (out_len) *out_len = total;
  if (n_members) *n_members = (uint32_t)jobs.size();
  if (jobs.empty()) return GZ_E_HEADER;
  if (d_out && total > out_cap) {
    snprintf(g_err, sizeof(g_err), "output needs %llu bytes", (unsigned long long)total);
    return GZ_E_CAPACITY;
  }
  gz_plan_t p = new (std::nothrow) gz_plan_s();
  if (!p) return GZ_E_ARG;
  fill_defaults(p, opts);
  if (!valid_opts(p)) {
    gz_plan_destroy(p);
    return GZ_E_ARG;
  }
  p->jobs = jobs;
  p->pre = pre;
  const int r = plan_common(p);
  if (r != GZ_OK) {
    gz_plan_destroy(p);
    return r;
  }
  (void)hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
  if (p->opts.timing)
    for (int i = 0; i <= GZ_N_PASSES; i++) (void)hipEventCreate(&p->pass_ev[i]);
  *plan = p;
  return GZ_OK;
}

int gz_find_blocks(gz_plan_t p, void *d_ws, size_t ws_bytes, void *stream) {
  if (!p || !p->probe) return GZ_E_ARG;
  return launch(p, (uint8_t *)d_ws, ws_bytes, (hipStream_t)stream);
}

int gz_probe_starts(gz_plan_t p, uint64_t *start_bits, uint32_t *n_retries) {
  if (!p || !p->probe || !start_bits) return GZ_E_ARG;
  const int r = fetch_chunks(p);
  if (r != GZ_OK) return r;
  for (size_t f = 0; f < p->files.size(); f++) {
    const ChunkState &c = p->cst[p->files[f].first_chunk];
    const bool ok = c.start != NONE && c.status == ST_OK && !(c.flags & CS_UNCONFIRMED);
    start_bits[f] = ok ? c.start : NONE;
    if (n_retries) n_retries[f] = c.retries;
  }
  return GZ_OK;
}

int gz_count_byte(const void *d_buf, uint64_t n, uint32_t value, uint64_t first, uint64_t window,
                  uint64_t *d_counts, uint64_t n_counts, void *stream) {
  if ((!d_buf && n) || value > 255 || window == 0 || (!d_counts && n_counts)) return GZ_E_ARG;
  hipError_t e = gzk_count_byte((const uint8_t *)d_buf, n, value, first, window, (unsigned long long *)d_counts,
                                n_counts, (hipStream_t)stream);
  return e == hipSuccess ? GZ_OK : hip_fail(e, "count");
}

uint64_t gz_extract_dna_ws(uint64_t n) { return gzk_dna_ws(n); }

int gz_extract_dna(const void *d_buf, uint64_t n, uint32_t elem_bytes, uint32_t marker, uint32_t min_len,
                   gz_dna_seq *d_seqs, uint64_t max_seqs, uint64_t *d_n_seqs, const uint64_t *d_bounds,
                   uint32_t n_ranges, uint32_t threshold, uint32_t *d_range_stats, void *d_ws, size_t ws_bytes,
                   void *stream) {
  const bool bad_marker = elem_bytes == 1 && (marker > 255 || marker == '\n' || marker == 'A' || marker == 'C' ||
                                              marker == 'G' || marker == 'T' || marker == 'N');
  if ((elem_bytes != 1 && elem_bytes != 2) || n >= (1ull << 32) || bad_marker || (!d_buf && n) || !d_n_seqs ||
      (!d_seqs && max_seqs) || (n_ranges && (!d_bounds || !d_range_stats)) || !d_ws || ((uintptr_t)d_ws & 255u)) {
    snprintf(g_err, sizeof(g_err), "gz_extract_dna: invalid argument");
    return GZ_E_ARG;
  }
  if (ws_bytes < gzk_dna_ws(n)) return GZ_E_CAPACITY;
  hipError_t e = gzk_dna(d_buf, n, elem_bytes, marker, min_len, d_seqs, max_seqs, d_n_seqs, d_bounds, n_ranges,
                         threshold, d_range_stats, (uint8_t *)d_ws, (hipStream_t)stream);
  return e == hipSuccess ? GZ_OK : hip_fail(e, "extract");
}

int gz_plan_info(gz_plan_t p, gz_info *info) {
  if (!p || !info) return GZ_E_ARG;
  memset(info, 0, sizeof(*info));
  info->ws_bytes = p->lay.total;
  info->payload_start = p->files[0].payload_bit / 8;
  info->payload_end = p->files[0].trailer_byte;
  info->n_files = (uint32_t)p->files.size();
  info->n_chunks = (uint32_t)p->chunks.size();
  info->crc32 = p->files[0].crc;
  info->isize = p->files[0].isize;
  return GZ_OK;
}

static int launch(gz_plan_t p, uint8_t *ws, size_t ws_bytes, hipStream_t st) {
  if (!ws || ws_bytes < p->lay.total || ((uintptr_t)ws & 255u)) {
    snprintf(g_err, sizeof(g_err), "workspace needs %llu bytes, 256-byte aligned",
             (unsigned long long)p->lay.total);
    return ws && ws_bytes < p->lay.total ? GZ_E_CAPACITY : GZ_E_ARG;
  }
  const Layout &L = p->lay;
  const uint32_t F = (uint32_t)p->files.size(), N = (uint32_t)p->chunks.size();
  if (p->upload_pending) {
    (void)hipEventSynchronize(p->upload_done);
    p->upload_pending = false;
  }
  if (p->capturing && p->opts.timing) return GZ_E_ARG;
  // CRC units of each file's output capacity, in file order
  uint64_t crc_units = 0;
  for (FileDesc &fd : p->files) {
    fd.crc_unit0 = crc_units;
    crc_units += fd.out ? (fd.out_cap + CRC_UNIT - 1) / CRC_UNIT : 0;
  }
  memcpy(p->pinned + L.files_off, p->files.data(), F * sizeof(FileDesc));
  memcpy(p->pinned + L.chunks_off, p->chunks.data(), (size_t)N * sizeof(ChunkDesc));
  memcpy(p->pinned + L.order_off, p->order.data(), (size_t)N * 4);
  if (!p->scan_list.empty()) memcpy(p->pinned + p->scan_off, p->scan_list.data(), p->scan_list.size() * 4);
  crc_xpow_table((uint32_t *)(p->pinned + L.crc_off));
  int ev = 0;
  auto mark = [&]() {
    if (p->opts.timing && ev <= GZ_N_PASSES) (void)hipEventRecord(p->pass_ev[ev++], st);
  };
  mark();
  hipError_t e = hipMemcpyAsync(ws, p->pinned, L.table_bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "job table upload");
  if (!p->capturing) {
    // the pinned table may be rewritten by the next call once this copy is done
    (void)hipEventRecord(p->upload_done, st);
    p->upload_pending = true;
  }

  const FileDesc *files = (const FileDesc *)(ws + L.files_off);
  const ChunkDesc *chunks = (const ChunkDesc *)(ws + L.chunks_off);
  const uint32_t *order = (const uint32_t *)(ws + L.order_off);
  const uint32_t *scan = (const uint32_t *)(ws + p->scan_off);
  ChunkState *cs = (ChunkState *)(ws + L.cstate_off);
  FileState *fs = (FileState *)(ws + L.fstate_off);
  Counters *ctr = (Counters *)(ws + L.counters_off);
  uint64_t *tiles = (uint64_t *)(ws + L.tiles_off);
  uint32_t *acc_pos = (uint32_t *)(ws + L.acc_off);
  AccEntry *acc = (AccEntry *)(ws + align_up(L.acc_off + ((uint64_t)N + 1) * 4, 256));
  uint8_t *wins = ws + L.win_off;
  uint16_t *pool = (uint16_t *)(ws + L.sym_off);

  uint32_t grid = (uint32_t)std::min<uint64_t>(N, decode_slots(p));
  if (grid == 0) grid = 1;

  mark();
  if ((e = gzk_init(cs, N, fs, F, ctr, st)) != hipSuccess) return hip_fail(e, "init");
  mark();
  if ((e = gzk_scan(files, chunks, cs, scan, (uint32_t)p->scan_list.size(), p->groups, st)) != hipSuccess)
    return hip_fail(e, "scan");
  mark();
  if ((e = gzk_capacity(F, files, (ChunkDesc *)(ws + L.chunks_off), cs, p->opts.sym_factor, st)) != hipSuccess)
    return hip_fail(e, "capacity");
  mark();
  if ((e = gzk_inflate((int)p->win, (p->opts.start_types & GZ_START_STORED) ? 1u : 0u, grid, files, chunks, cs, order,
                       N, ctr, pool, st)) != hipSuccess)
    return hip_fail(e, "inflate");
  mark();
  if ((e = gzk_confirm((int)p->win, grid, files, chunks, cs, N, ctr, pool, p->opts.confirm_decode, st)) != hipSuccess)
    return hip_fail(e, "confirm");
  mark();
  if ((e = gzk_redo((int)p->win, grid, files, chunks, cs, N, ctr, pool, st)) != hipSuccess) return hip_fail(e, "redo");
  mark();
  if (p->probe) {
    // block-start probes end with their confirmed starts
    p->timed = false;
    p->ws = ws;
    p->stream = st;
    p->launched = true;
    p->fetched = false;
    return GZ_OK;
  }
  if ((e = gzk_stitch((int)p->win, grid, files, chunks, cs, N, ctr, pool, st)) != hipSuccess)
    return hip_fail(e, "stitch");
  mark();
  if ((e = gzk_finalize((int)p->win, F, files, chunks, cs, fs, pool, st)) != hipSuccess) return hip_fail(e, "finalize");
  mark();
  if ((e = gzk_tilescan(chunks, cs, fs, N, tiles, acc_pos, acc, st)) != hipSuccess) return hip_fail(e, "tilescan");
  mark();
  if ((e = gzk_propagate(N, acc_pos, acc, wins, pool, (uint16_t *)(ws + L.maps_off), ws + L.segwin_off, st)) !=
      hipSuccess)
    return hip_fail(e, "propagate");
  mark();
  if ((e = gzk_translate((uint32_t)p->n_cu * 8, files, chunks, cs, fs, tiles, N, wins, pool, ctr, st)) !=
      hipSuccess)
    return hip_fail(e, "translate");
  mark();
  if ((e = gzk_crc(F, files, fs, (const uint32_t *)(ws + L.crc_off), crc_units, st)) != hipSuccess)
    return hip_fail(e, "crc");
  mark();
  if (p->capturing) return GZ_OK;
  p->timed = p->opts.timing != 0;
  p->ws = ws;
  p->stream = st;
  p->launched = true;
  p->fetched = false;
  return GZ_OK;
}

static void drop_graph(gz_plan_t p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  p->graph_ws = nullptr;
  p->graph_out.clear();
}

int gz_decompress(gz_plan_t p, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes, void *stream) {
  if (!p || p->files.size() != 1 || p->probe) return GZ_E_ARG;
  if (!d_out && out_cap) return GZ_E_ARG;
  p->files[0].out = (uint8_t *)d_out;
  p->files[0].out_cap = d_out ? out_cap : 0;
  return launch(p, (uint8_t *)d_ws, ws_bytes, (hipStream_t)stream);
}

static_assert(SCRATCH_BYTES == GZ_SCRATCH_BYTES, "static workspace size");

int gz_decompress_static(gz_plan_t p, void *d_out, size_t out_cap, void *stream) {
  if (!p || p->files.size() != 1 || p->probe || p->seg.on) return GZ_E_ARG;
  if (!d_out && out_cap) return GZ_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
    snprintf(g_err, sizeof(g_err), "the plan belongs to device %d, the current device is %d", p->device, dev);
    return GZ_E_ARG;
  }
  if (p->lay.total > SCRATCH_BYTES) {
    snprintf(g_err, sizeof(g_err), "workspace of %llu bytes exceeds the static workspace of %llu bytes",
             (unsigned long long)p->lay.total, (unsigned long long)SCRATCH_BYTES);
    return GZ_E_CAPACITY;
  }
  void *ws = nullptr;
  const hipError_t e = gzk_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "static workspace address");
  p->files[0].out = (uint8_t *)d_out;
  p->files[0].out_cap = d_out ? out_cap : 0;
  return launch(p, (uint8_t *)ws, SCRATCH_BYTES, (hipStream_t)stream);
}

int gz_decompress_batch(gz_plan_t p, void *d_ws, size_t ws_bytes, void *stream) {
  if (!p || p->probe) return GZ_E_ARG;
  return launch(p, (uint8_t *)d_ws, ws_bytes, (hipStream_t)stream);
}

int gz_decompress_graph(gz_plan_t p, void *d_ws, size_t ws_bytes, void *stream) {
  if (!p || !stream || p->opts.timing || p->probe) return GZ_E_ARG;
  if (!d_ws || ws_bytes < p->lay.total || ((uintptr_t)d_ws & 255u)) {
    snprintf(g_err, sizeof(g_err), "workspace needs %llu bytes, 256-byte aligned",
             (unsigned long long)p->lay.total);
    return d_ws && ws_bytes < p->lay.total ? GZ_E_CAPACITY : GZ_E_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::pair<uint8_t *, uint64_t>> outs;
  for (const FileDesc &f : p->files) outs.emplace_back(f.out, f.out_cap);
  if (!p->graph_exec || p->graph_ws != (uint8_t *)d_ws || p->graph_out != outs) {
    drop_graph(p);
    // the table is written once here and only read by the replays
    if (p->upload_pending) {
      (void)hipEventSynchronize(p->upload_done);
      p->upload_pending = false;
    }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    p->capturing = true;
    const int r = launch(p, (uint8_t *)d_ws, ws_bytes, st);
    p->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (r != GZ_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    p->graph = g;
    e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(p);
      return hip_fail(e, "graph instantiate");
    }
    p->graph_ws = (uint8_t *)d_ws;
    p->graph_out = outs;
  }
  hipError_t e = hipGraphLaunch(p->graph_exec, st);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  p->timed = false;
  p->ws = (uint8_t *)d_ws;
  p->stream = st;
  p->launched = true;
  p->fetched = false;
  return GZ_OK;
}

static int fetch(gz_plan_t p) {
  if (!p->launched) return GZ_E_NOT_READY;
  if (p->fetched) return GZ_OK;
  // wait with a deadline (GZGPU_TIMEOUT_S, default 120 s) instead of blocking
  // forever on a stream that does not finish
  double limit = 120.0;
  if (const char *t = getenv("GZGPU_TIMEOUT_S")) limit = atof(t);
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e;
  for (;;) {
    e = hipStreamQuery(p->stream);
    if (e != hipErrorNotReady) break;
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (el > limit) {
      snprintf(g_err, sizeof(g_err), "the stream did not finish within %.0f s", limit);
      return GZ_E_HIP;
    }
    // short polls for the first second, so that a finished run is seen
    // within tens of microseconds
    std::this_thread::sleep_for(std::chrono::microseconds(el < 1.0 ? 20 : 1000));
  }
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  const uint32_t F = (uint32_t)p->files.size();
  p->fst.resize(F);
  e = copy_to_host(p->fst.data(), p->ws + p->lay.fstate_off, F * sizeof(FileState), p->stream);
  if (e != hipSuccess) return hip_fail(e, "reading file state");
  p->fetched = true;
  p->fetched_chunks = false;
  return GZ_OK;
}

// fetch(), and the per-chunk states and chunk table (read only by the calls
// that report per-chunk data, and when a chunk overflowed its capacity).
static int fetch_chunks(gz_plan_t p) {
  int r = fetch(p);
  if (r != GZ_OK) return r;
  if (p->fetched_chunks) return GZ_OK;
  const uint32_t N = (uint32_t)p->chunks.size();
  p->cst.resize(N);
  hipError_t e = copy_to_host(p->cst.data(), p->ws + p->lay.cstate_off, (size_t)N * sizeof(ChunkState), p->stream);
  if (e != hipSuccess) return hip_fail(e, "reading chunk state");
  p->cdev.resize(N);
  e = copy_to_host(p->cdev.data(), p->ws + p->lay.chunks_off, (size_t)N * sizeof(ChunkDesc), p->stream);
  if (e != hipSuccess) return hip_fail(e, "reading chunk table");
  p->fetched_chunks = true;
  return GZ_OK;
}

// Symbol factor that covers the worst overflowing chunk of a file, with room.
static uint64_t needed_factor(gz_plan_t p, int file) {
  const FileDesc &fd = p->files[file];
  double worst = 0;
  for (uint32_t c = fd.first_chunk; c < fd.first_chunk + fd.n_chunks; c++)
    if (p->cst[c].flags & CS_OVERFLOW) {
      const ChunkDesc &d = p->cdev[c];
      const double span = d.sym_cap > SYM_SLACK ? (double)(d.sym_cap - SYM_SLACK) / p->opts.sym_factor : 1.0;
      worst = std::max(worst, (double)p->cst[c].needed / span);
    }
  return (uint64_t)(worst * 1.25) + 1;
}

int gz_result_get(gz_plan_t p, int file, gz_result *res) {
  if (!p || !res || file < 0 || file >= (int)p->files.size()) return GZ_E_ARG;
  int r = fetch(p);
  if (r != GZ_OK) return r;
  const FileState &s = p->fst[file];
  const FileDesc &fd = p->files[file];
  memset(res, 0, sizeof(*res));
  res->status = s.status;
  res->n_chunks = fd.n_chunks;
  res->out_len = s.out_len;
  res->out_needed = s.out_needed;
  res->n_nonempty = s.n_nonempty;
  res->n_repairs = s.n_repairs;
  res->n_extended = s.n_extended;
  res->n_retries = s.n_retries;
  res->n_syms = s.n_syms;
  res->n_placeholders = s.n_placeholders;
  res->n_blocks = s.n_blocks;
  res->crc32 = s.crc_out;
  res->inflate_waves = (uint32_t)std::min<uint64_t>(p->chunks.size(), decode_slots(p));
  if (s.overflow) {
    // the workspace of a plan whose symbol factor covers the worst chunk
    r = fetch_chunks(p);
    if (r != GZ_OK) return r;
    const uint64_t f2 = needed_factor(p, file);
    res->ws_needed = p->lay.total + 2 * (f2 > p->opts.sym_factor ? f2 - p->opts.sym_factor : 1) * p->span[file];
  }
  return GZ_OK;
}

int gz_chunk_table(gz_plan_t p, int file, uint64_t *start, uint64_t *cand, uint64_t *end, uint64_t *len,
                   uint64_t *out_off, int32_t *status, uint32_t *flags) {
  if (!p || file < 0 || file >= (int)p->files.size()) return GZ_E_ARG;
  int r = fetch_chunks(p);
  if (r != GZ_OK) return r;
  const FileDesc &fd = p->files[file];
  for (uint32_t i = 0; i < fd.n_chunks; i++) {
    const ChunkState &s = p->cst[fd.first_chunk + i];
    if (start) start[i] = s.start;
    if (cand) cand[i] = s.found;
    if (end) end[i] = s.end;
    if (len) len[i] = s.len;
    if (out_off) out_off[i] = s.out_off;
    if (status) status[i] = s.status;
    if (flags) flags[i] = s.flags;
  }
  return GZ_OK;
}

int gz_chunk_stats(gz_plan_t p, int file, uint64_t *n_syms, uint64_t *n_placeholders, uint32_t *n_blocks,
                   uint64_t *scan_cand, uint32_t *stage1, uint32_t *stage2, uint32_t *trial_rej,
                   uint32_t *confirm_rej) {
  if (!p || file < 0 || file >= (int)p->files.size()) return GZ_E_ARG;
  int r = fetch_chunks(p);
  if (r != GZ_OK) return r;
  const FileDesc &fd = p->files[file];
  for (uint32_t i = 0; i < fd.n_chunks; i++) {
    const ChunkState &s = p->cst[fd.first_chunk + i];
    const bool ne = s.start != NONE;
    if (n_syms) n_syms[i] = ne ? s.n_syms : 0;
    if (n_placeholders) n_placeholders[i] = ne ? s.n_placeholders : 0;
    if (n_blocks) n_blocks[i] = ne ? s.n_blocks : 0;
    if (scan_cand) scan_cand[i] = s.cand;
    if (stage1) stage1[i] = s.stage1;
    if (stage2) stage2[i] = s.stage2;
    if (trial_rej) trial_rej[i] = s.trial_rej;
    if (confirm_rej) confirm_rej[i] = s.confirm_rej;
  }
  return GZ_OK;
}

int gz_debug_layout(gz_plan_t p, int file, uint64_t *sym_off, uint64_t *win_index, void **sym_base, void **win_base) {
  if (!p || file < 0 || file >= (int)p->files.size() || !p->launched) return GZ_E_ARG;
  int r = fetch_chunks(p);
  if (r != GZ_OK) return r;
  const FileDesc &fd = p->files[file];
  for (uint32_t i = 0; i < fd.n_chunks; i++) {
    if (sym_off) sym_off[i] = p->cdev[fd.first_chunk + i].sym_off;
    if (win_index) win_index[i] = fd.first_chunk + i;
  }
  if (sym_base) *sym_base = p->ws + p->lay.sym_off;
  if (win_base) *win_base = p->ws + p->lay.win_off;
  return GZ_OK;
}

int gz_pass_times(gz_plan_t p, float *ms, int n) {
  if (!p || !ms || n < 0) return GZ_E_ARG;
  if (!p->launched || !p->timed) return GZ_E_NOT_READY;
  int r = fetch(p);
  if (r != GZ_OK) return r;
  int k = 0;
  for (; k < n && k < GZ_N_PASSES; k++) {
    float t = 0.f;
    hipError_t e = hipEventElapsedTime(&t, p->pass_ev[k], p->pass_ev[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "event timing");
    ms[k] = t;
  }
  return k;
}

const char *gz_pass_name(int i) {
  static const char *names[GZ_N_PASSES] = {"upload",   "init",     "scan",      "capacity",  "inflate",
                                           "confirm",  "redo",     "stitch",    "finalize",  "tilescan",
                                           "propagate", "translate", "crc"};
  return i >= 0 && i < GZ_N_PASSES ? names[i] : "";
}

void gz_plan_destroy(gz_plan_t p) {
  if (!p) return;
  drop_graph(p);
  if (p->upload_pending) (void)hipEventSynchronize(p->upload_done);
  if (p->upload_done) (void)hipEventDestroy(p->upload_done);
  for (int i = 0; i <= GZ_N_PASSES; i++)
    if (p->pass_ev[i]) (void)hipEventDestroy(p->pass_ev[i]);
  if (p->pinned) (void)hipHostFree(p->pinned);
  delete p;
}

const char *gz_strerror(int code) {
  switch (code) {
    case GZ_OK: return "ok";
    case GZ_E_ARG: return g_err[0] ? g_err : "invalid argument";
    case GZ_E_HEADER: return "invalid gzip header";
    case GZ_E_UNSUPPORTED: return "unsupported input (data after the first gzip member)";
    case GZ_E_DATA: return "invalid compressed data";
    case GZ_E_CAPACITY: return "output or workspace too small";
    case GZ_E_SIZE: return "decompressed size does not match the trailer";
    case GZ_E_CRC: return "CRC-32 of the output does not match the trailer";
    case GZ_E_HIP: return g_err[0] ? g_err : "HIP runtime error";
    case GZ_E_NOT_READY: return "no decompression launched on this plan";
    default: return "unknown error";
  }
}

// Autotuner: candidate (chunk size, LDS ring) pairs timed on the caller's
// input; the choice is cached per (device, size class, ratio class).
namespace {
const uint64_t k_tune_chunks[] = {32ull << 10, 40ull << 10, 64ull << 10, 128ull << 10, 256ull << 10, 1ull << 20};
const uint32_t k_tune_rings[] = {512, 1024, 2048};
}  // namespace

int gz_autotune(const void *d_comp, size_t comp_len, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes,
                void *stream, gz_opts *best, uint64_t *ws_max) {
  if (!d_comp || comp_len == 0 || !best) return GZ_E_ARG;
  const gz_opts base = *best;
  // candidates and the workspace the largest one needs
  std::vector<gz_opts> cand;
  uint64_t need = 0;
  uint32_t isize = 0;
  uint64_t payload = 0;
  for (uint64_t cb : k_tune_chunks) {
    for (uint32_t ring : k_tune_rings) {
      gz_opts o = base;
      o.chunk_bytes = cb;
      o.window_syms = ring;
      o.timing = 0;
      o.tuned = 0;
      gz_plan_t pl = nullptr;
      int r = gz_plan(&pl, d_comp, comp_len, 0, &o);
      if (r != GZ_OK) return r;
      gz_info inf;
      gz_plan_info(pl, &inf);
      gz_plan_destroy(pl);
      payload = inf.payload_end - inf.payload_start;
      isize = inf.isize;
      // at least two chunks, except for inputs below the smallest chunk size
      if (cb != k_tune_chunks[0] && cb * 2 > payload) continue;
      need = std::max<uint64_t>(need, inf.ws_bytes);
      cand.push_back(o);
    }
  }
  if (ws_max) *ws_max = need;
  if (!d_ws) return GZ_OK;  // query only
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = tune_key(dev, comp_len, payload, isize);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *best = it->second;
      best->timing = base.timing;
      return GZ_OK;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best_ms = -1.f;
  int last = GZ_E_CAPACITY;
  for (const gz_opts &o : cand) {
    gz_plan_t pl = nullptr;
    int r = gz_plan(&pl, d_comp, comp_len, 0, &o);
    if (r != GZ_OK) {
      last = r;
      continue;
    }
    gz_info inf;
    gz_plan_info(pl, &inf);
    float ms = -1.f;
    if (inf.ws_bytes <= ws_bytes) {
      gz_result res;
      r = gz_decompress(pl, d_out, out_cap, d_ws, ws_bytes, st);  // warm
      if (r == GZ_OK) r = gz_result_get(pl, 0, &res);
      if (r == GZ_OK && res.status == GZ_OK) {
        (void)hipEventRecord(e0, st);
        r = gz_decompress(pl, d_out, out_cap, d_ws, ws_bytes, st);
        (void)hipEventRecord(e1, st);
        if (r == GZ_OK) r = gz_result_get(pl, 0, &res);
        if (r == GZ_OK && res.status == GZ_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.f;
      } else if (r == GZ_OK) {
        r = res.status;
      }
      last = r;
    }
    gz_plan_destroy(pl);
    if (ms > 0.f && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      *best = o;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms < 0.f) return last != GZ_OK ? last : GZ_E_CAPACITY;
  best->timing = base.timing;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = *best;
  return GZ_OK;
}

int gz_device_info(int dev, int *n_cu, int *lds_bytes) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "device properties");
  if (n_cu) *n_cu = prop.multiProcessorCount;
  if (lds_bytes) *lds_bytes = (int)prop.maxSharedMemoryPerMultiProcessor;
  return GZ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Bounded-memory streaming: one plan per segment (see gz_stream_open).
// ---------------------------------------------------------------------------

struct gz_stream_s {
  gz_job job{};
  gz_opts opts{};
  uint64_t seg_bytes = 0;
  int64_t h = 0;
  uint32_t crc = 0, isize = 0;
  uint8_t *h_win = nullptr;  // carried window: 32 KiB of pinned host memory, copied into each segment's workspace
  // position after the last finished segment: bytes of all members, and of
  // the current member (its CRC-32, its real history in the window)
  uint64_t bit = 0, out_total = 0, member_out = 0;
  uint32_t crc_run = 0, valid = 0, member = 0;
  bool done = false;
  gz_plan_t cur = nullptr;   // plan of the segment in flight, re-planned in place for the next
  bool pending = false;
  bool inside = false;       // opened at a block inside the member (gz_stream_open_at)
  uint64_t info_ws = 0, info_out = 0;  // sizes for any segment at the current symbol factor (0: not known)
};

// Plan a segment into *io (created when null, else re-planned in place so
// its pinned table is reused).
static int segment_plan(gz_stream_t s, uint64_t start_bit, uint32_t win_valid, void *d_out, uint64_t out_cap,
                        gz_plan_t *io) {
  gz_plan_t p = *io;
  const bool fresh = p == nullptr;
  if (fresh) {
    p = new (std::nothrow) gz_plan_s();
    if (!p) return GZ_E_ARG;
  } else {
    if (p->upload_pending) {
      (void)hipEventSynchronize(p->upload_done);
      p->upload_pending = false;
    }
    p->launched = false;
    p->fetched = false;
  }
  fill_defaults(p, &s->opts, fresh);
  p->seg.on = true;
  p->seg.start_bit = start_bit;
  p->seg.stop_bit = start_bit + 8 * s->seg_bytes;
  p->seg.out_before = s->member_out;
  p->seg.crc_in = s->crc_run;
  p->seg.win_valid = win_valid;
  p->seg.mode = (s->inside ? FD_NOCHECK : 0u) | FD_MEMBERS;
  p->seg.h = s->h;
  p->seg.crc = s->crc;
  p->seg.isize = s->isize;
  gz_job j = s->job;
  j.d_out = d_out;
  j.out_cap = out_cap;
  p->jobs.assign(1, j);
  const int r = plan_common(p);
  if (r != GZ_OK) {
    gz_plan_destroy(p);
    *io = nullptr;
    return r;
  }
  if (fresh) (void)hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming);
  *io = p;
  return GZ_OK;
}

// Workspace and output sizes of a full segment that starts from a carried
// window (the largest layout), at the current symbol factor.
static int stream_sizes(gz_stream_t s) {
  gz_plan_t p = nullptr;
  const int r = segment_plan(s, 8ull * (uint64_t)s->h, WINDOW, nullptr, 0, &p);
  if (r != GZ_OK) return r;
  s->info_ws = p->lay.total;
  s->info_out = p->files[0].pool_elems;
  gz_plan_destroy(p);
  return GZ_OK;
}

extern "C" {

int gz_stream_open(gz_stream_t *stream, const void *d_comp, size_t comp_len, uint64_t segment_bytes,
                   const gz_opts *opts) {
  if (!stream || !d_comp || comp_len == 0) return GZ_E_ARG;
  *stream = nullptr;
  gz_stream_t s = new (std::nothrow) gz_stream_s();
  if (!s) return GZ_E_ARG;
  if (opts) s->opts = *opts;
  s->opts.timing = 0;
  if (!s->opts.sym_factor) s->opts.sym_factor = 8;
  s->seg_bytes = segment_bytes ? segment_bytes : (256ull << 20);
  s->job.d_comp = d_comp;
  s->job.comp_len = comp_len;
  int r = read_member(s->job, 0, &s->h, &s->crc, &s->isize);
  if (r == GZ_OK) {
    hipError_t e = hipHostMalloc((void **)&s->h_win, WINDOW, hipHostMallocDefault);
    if (e != hipSuccess) r = hip_fail(e, "stream window buffer (pinned host memory)");
    else memset(s->h_win, 0, WINDOW);
  }
  if (r != GZ_OK) {
    gz_stream_destroy(s);
    return r;
  }
  s->bit = 8ull * (uint64_t)s->h;
  *stream = s;
  return GZ_OK;
}

int gz_stream_get_info(gz_stream_t s, gz_stream_info *info) {
  if (!s || !info) return GZ_E_ARG;
  memset(info, 0, sizeof(*info));
  if (!s->info_ws) {
    const int r = stream_sizes(s);
    if (r != GZ_OK) return r;
  }
  info->ws_bytes = s->info_ws;
  info->out_bytes = s->info_out;
  info->segment_bytes = s->seg_bytes;
  info->payload_start = (uint64_t)s->h;
  info->payload_end = s->job.comp_len - 8;
  info->crc32 = s->crc;
  info->isize = s->isize;
  return GZ_OK;
}

int gz_stream_next(gz_stream_t s, void *d_out, size_t out_cap, void *d_ws, size_t ws_bytes, void *hip_stream) {
  if (!s || s->done || s->pending || !d_out || out_cap == 0) return GZ_E_ARG;
  const uint32_t wv = s->inside ? WINDOW : (uint32_t)std::min<uint64_t>(s->member_out, WINDOW);
  int r = segment_plan(s, s->bit, wv, d_out, out_cap, &s->cur);
  if (r != GZ_OK) return r;
  gz_plan_t p = s->cur;
  uint8_t *ws = (uint8_t *)d_ws;
  hipStream_t st = (hipStream_t)hip_stream;
  if (!ws || ws_bytes < p->lay.total || ((uintptr_t)ws & 255u)) {
    snprintf(g_err, sizeof(g_err), "workspace needs %llu bytes, 256-byte aligned",
             (unsigned long long)p->lay.total);
    return ws && ws_bytes < p->lay.total ? GZ_E_CAPACITY : GZ_E_ARG;
  }
  // the first chunk's window slot holds the carried window (nothing else
  // writes that slot before window propagation reads it); the pinned copy is
  // rewritten only after this segment has finished
  uint8_t *slot = ws + p->lay.win_off + (uint64_t)p->files[0].first_chunk * WINDOW;
  hipError_t e;
  if (wv > 0 && (e = hipMemcpyAsync(slot, s->h_win, WINDOW, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "carried window");
  r = launch(p, ws, ws_bytes, st);
  if (r == GZ_OK) {
    // the next window: the last 32 KiB of (carried window ++ this output),
    // into the workspace's carry area (read back by gz_stream_wait)
    e = gzk_carry((const FileDesc *)(ws + p->lay.files_off), (const FileState *)(ws + p->lay.fstate_off), slot,
                  ws + p->lay.carry_off, st);
    if (e != hipSuccess) r = hip_fail(e, "carry");
  }
  if (r != GZ_OK) return r;
  s->pending = true;
  return GZ_OK;
}

int gz_stream_wait(gz_stream_t s, gz_segment_result *res) {
  if (!s || !res || !s->cur || !s->pending) return GZ_E_ARG;
  gz_result g;
  int r = gz_result_get(s->cur, 0, &g);
  if (r != GZ_OK) return r;
  s->pending = false;
  const FileState &fst = s->cur->fst[0];
  memset(res, 0, sizeof(*res));
  res->status = g.status;
  res->out_len = g.out_len;
  res->start_bit = s->bit;
  res->end_bit = fst.end_bit;
  res->n_chunks = g.n_chunks;
  res->n_repairs = g.n_repairs;
  res->n_retries = g.n_retries;
  res->out_needed = g.out_needed;
  res->member = s->member;
  if (g.status == GZ_OK) {
    // the window after this segment, from the workspace's carry area
    hipError_t e = copy_to_host(s->h_win, s->cur->ws + s->cur->lay.carry_off, WINDOW, s->cur->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the carried window");
    s->bit = fst.end_bit;
    s->out_total += g.out_len;
    s->member_out += g.out_len;
    s->crc_run = g.crc32;
    s->valid = s->inside ? WINDOW : (uint32_t)std::min<uint64_t>(s->member_out, WINDOW);
    if (fst.is_final) {
      // the member is done; more bytes after its trailer are the next member
      res->member_done = 1;
      const uint64_t te = ((fst.end_bit + 7) >> 3) + 8;
      s->done = true;
      if (te < s->job.comp_len) {
        gz_job nj = s->job;
        nj.d_comp = (const uint8_t *)s->job.d_comp + te;
        nj.comp_len = s->job.comp_len - te;
        int64_t h = 0;
        uint32_t c = 0, z = 0;
        const int hr = nj.comp_len >= 18 ? read_member(nj, 0, &h, &c, &z) : GZ_E_HEADER;
        if (hr != GZ_OK) {
          res->status = hr == GZ_E_HIP ? GZ_E_HIP : GZ_E_HEADER;
        } else {
          s->done = false;
          s->member++;
          s->bit = 8 * (te + (uint64_t)h);
          s->member_out = 0;
          s->crc_run = 0;
          s->valid = 0;
          s->inside = false;
        }
      }
    }
  } else if (g.status == GZ_E_CAPACITY && fst.overflow) {
    // symbols overflowed: later plans use a factor that covers them
    const uint64_t f2 = needed_factor(s->cur, 0);
    s->opts.sym_factor = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(f2, 2ull * s->opts.sym_factor), 1u << 20);
    s->info_ws = 0;
    gz_stream_info info;
    if (gz_stream_get_info(s, &info) == GZ_OK) res->ws_needed = info.ws_bytes;
  }
  res->done = s->done ? 1u : 0u;
  res->out_total = s->out_total;
  res->crc32 = g.status == GZ_OK ? g.crc32 : s->crc_run;
  return GZ_OK;
}

int gz_stream_checkpoint(gz_stream_t s, gz_checkpoint *cp) {
  if (!s || !cp || s->pending) return GZ_E_ARG;
  memset(cp, 0, sizeof(*cp));
  cp->bit = s->bit;
  cp->out_total = s->out_total;
  cp->member_out = s->member_out;
  cp->member = s->member;
  cp->crc32 = s->crc_run;
  cp->valid = s->valid;
  cp->done = s->done ? 1u : 0u;
  cp->flags = s->inside ? 1u : 0u;
  if (s->valid > 0) memcpy(cp->window, s->h_win, WINDOW);
  return GZ_OK;
}

int gz_stream_resume(gz_stream_t s, const gz_checkpoint *cp) {
  if (!s || !cp || s->pending) return GZ_E_ARG;
  const uint64_t lo = 8ull * (uint64_t)s->h, hi = 8ull * (s->job.comp_len - 8);
  const bool inside = (cp->flags & 1u) != 0;
  if (cp->bit < lo || cp->bit > hi || cp->valid > WINDOW || (cp->flags & ~1u) || cp->member_out > cp->out_total ||
      cp->valid != (inside ? WINDOW : (uint32_t)std::min<uint64_t>(cp->member_out, WINDOW)))
    return GZ_E_ARG;
  if (cp->valid > 0) memcpy(s->h_win, cp->window, WINDOW);
  s->bit = cp->bit;
  s->out_total = cp->out_total;
  s->member_out = cp->member_out;
  s->member = cp->member;
  s->crc_run = cp->crc32;
  s->valid = cp->valid;
  s->done = cp->done != 0;
  s->inside = inside;
  return GZ_OK;
}

int gz_stream_open_at(gz_stream_t *stream, const void *d_comp, size_t comp_len, uint64_t block_bit, uint32_t marker,
                      uint64_t segment_bytes, const gz_opts *opts) {
  if (marker > 255) return GZ_E_ARG;
  int r = gz_stream_open(stream, d_comp, comp_len, segment_bytes, opts);
  if (r != GZ_OK) return r;
  gz_stream_t s = *stream;
  const uint64_t lo = 8ull * (uint64_t)s->h, hi = 8ull * (comp_len - 8);
  if (block_bit < lo || block_bit >= hi) {
    gz_stream_destroy(s);
    *stream = nullptr;
    return GZ_E_ARG;
  }
  // the undetermined context: 32768 copies of the marker
  memset(s->h_win, (int)marker, WINDOW);
  s->bit = block_bit;
  s->inside = true;
  s->valid = WINDOW;
  return GZ_OK;
}

void gz_stream_destroy(gz_stream_t s) {
  if (!s) return;
  if (s->cur) {
    if (s->pending) (void)hipStreamSynchronize(s->cur->stream);
    gz_plan_destroy(s->cur);
  }
  if (s->h_win) (void)hipHostFree(s->h_win);
  delete s;
}

// Concatenated members: a stream whose segments are whole members (the
// segment size is the whole input, and a segment ends at its member's final
// block), each decoded by the whole path, written back to back.
int gz_decompress_members(const void *d_comp, size_t comp_len, void *d_out, size_t out_cap, void *d_ws,
                          size_t ws_bytes, const gz_opts *opts, void *stream, uint64_t *out_len,
                          uint32_t *n_members, uint64_t *ws_needed) {
  if (out_len) *out_len = 0;
  if (n_members) *n_members = 0;
  if (!d_comp || comp_len == 0 || (d_ws && (!d_out || out_cap == 0))) return GZ_E_ARG;
  gz_stream_t s = nullptr;
  int r = gz_stream_open(&s, d_comp, comp_len, comp_len, opts);
  if (r != GZ_OK) return r;
  gz_stream_info info;
  r = gz_stream_get_info(s, &info);
  if (r == GZ_OK && ws_needed) *ws_needed = info.ws_bytes;
  if (r != GZ_OK || !d_ws) {
    gz_stream_destroy(s);
    return r;
  }
  uint64_t total = 0;
  uint32_t members = 0;
  // one segment per member; a capacity retry per segment at most
  for (uint64_t it = 0; it < 2 * (uint64_t)comp_len + 4; it++) {
    if (total >= out_cap) {
      snprintf(g_err, sizeof(g_err), "output full after %llu bytes", (unsigned long long)total);
      r = GZ_E_CAPACITY;
      break;
    }
    r = gz_stream_next(s, (uint8_t *)d_out + total, out_cap - total, d_ws, ws_bytes, stream);
    if (r != GZ_OK) break;
    gz_segment_result res;
    r = gz_stream_wait(s, &res);
    if (r != GZ_OK) break;
    if (res.status == GZ_E_CAPACITY && res.out_needed <= out_cap - total) {
      // more symbols than planned: the stream raised its factor; retry if
      // the workspace still suffices
      r = gz_stream_get_info(s, &info);
      if (r == GZ_OK && ws_needed) *ws_needed = info.ws_bytes;
      if (r == GZ_OK && info.ws_bytes <= ws_bytes) continue;
      if (r == GZ_OK) r = GZ_E_CAPACITY;
      break;
    }
    if (res.status == GZ_E_HEADER && res.member_done) {
      // the member is whole; the bytes after it are not a member
      total += res.out_len;
      members++;
      r = GZ_E_HEADER;
      break;
    }
    if (res.status != GZ_OK) {
      r = res.status;
      break;
    }
    total += res.out_len;
    if (res.member_done) members++;
    if (res.done) break;
  }
  if (out_len) *out_len = total;
  if (n_members) *n_members = members;
  gz_stream_destroy(s);
  return r;
}

}  // extern "C"
