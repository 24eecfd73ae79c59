// DNA-like sequences in partly undetermined text (Appendix B; Section VI-B's
// sequence-resolved blocks), on the device.
//
// The grammar T D+ (U+ D+)* T (D a nucleotide letter A C G T N, U an
// undetermined element, T a newline or an undetermined element), matched
// leftmost first, as long as possible, and resumed after the closing T.
// Every match lies inside one run of D and U elements (a maximal
// stretch of them) plus the element on each side, and a run holds at most
// one match:
//   - it opens at the newline before the run when the run starts with D and
//     that newline is still free, else at the first U followed by a D;
//   - it closes at the newline after the run when the run ends with D (and
//     that newline is consumed), at the first U after the run's last D when
//     the run ends with U, and otherwise at the first U after the last D
//     that a U follows;
//   - whatever is left of the run after the closing T holds no T D.
// The only coupling between runs is a single newline between two runs: the
// first run's match may consume it, and the second run then cannot open
// there.  With c_k = "run k consumed the newline after it", c_k = g_k(c_{k-1})
// for a map g_k of one bit, so the c's come from a scan of composed maps.
//
// Passes (one element = one byte, or one 16-bit symbol whose values of 256
// and above are placeholders):
//   k_dna_count   run starts per tile of DNA_TILE elements
//   k_dna_scan    exclusive prefix of per-group counts (one workgroup)
//   k_dna_runs    run start positions, in order
//   k_dna_props   one thread per run: walk the run, both possible matches
//                 (opened at the newline or at a U), its map g_k, and the
//                 composed map of each group of 256 runs
//   k_dna_chain   (one workgroup) the bit entering each group of runs
//   k_dna_select  the bit entering each run, the match taken, the length
//                 filter, accepted sequences per group
//   k_dna_write   sequences in order, per-range counts
//   k_dna_resolve the sequence-resolved flag of each range
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/gzgpu.h"
#include "gz_internal.h"

namespace gzgpu {

constexpr uint32_t DNA_TILE = 4096;   // elements per workgroup in the counting passes
constexpr uint32_t DNA_THREADS = 256;
constexpr uint32_t DNA_PER = DNA_TILE / DNA_THREADS;  // consecutive elements per thread

enum : uint32_t { DC_O = 0, DC_D = 1, DC_U = 2, DC_L = 3 };

// per run: the match opened at the newline before the run (A) and the one
// opened at the run's first U followed by D (B)
struct DnaRun {
  uint64_t a;        // first element of the run
  uint32_t lenA, nuA;
  uint32_t offB;     // B's first nucleotide, from a
  uint32_t lenB, nuB;
  uint32_t flags;
};
static_assert(sizeof(DnaRun) == 32, "run record");

enum : uint32_t {
  DR_A = 1u,          // A exists (starts with D after a newline, and closes)
  DR_B = 2u,          // B exists
  DR_CONSUMES = 4u,   // the match closes at the newline after the run
  DR_ADJ = 8u,        // the newline before the run closes the previous run when that run consumes it
  DR_G0 = 16u,        // g(0): consumed when the previous run did not consume the newline between them
  DR_G1 = 32u,        // g(1)
  DR_TAKE_A = 64u,
  DR_TAKE_B = 128u,
  DR_ACCEPT = 256u,   // taken and at least min_len long
};

__device__ __forceinline__ uint32_t byte_class(uint32_t b) {
  return (b == 'A' || b == 'C' || b == 'G' || b == 'T' || b == 'N') ? DC_D : (b == 0x0Au ? DC_L : DC_O);
}

template <int E>
__device__ __forceinline__ uint32_t elem_class(const void *buf, uint64_t i, uint32_t marker) {
  if (E == 2) {
    const uint32_t v = reinterpret_cast<const uint16_t *>(buf)[i];
    return v >= 256u ? DC_U : byte_class(v);
  }
  const uint32_t b = reinterpret_cast<const uint8_t *>(buf)[i];
  return b == marker ? DC_U : byte_class(b);
}

__device__ __forceinline__ bool in_run(uint32_t c) { return c == DC_D || c == DC_U; }

// map of one bit as two bits: bit 0 = f(0), bit 1 = f(1); (g after f)
__device__ __forceinline__ uint32_t map_then(uint32_t f, uint32_t g) {
  return ((g >> (f & 1u)) & 1u) | (((g >> ((f >> 1) & 1u)) & 1u) << 1);
}
constexpr uint32_t MAP_ID = 2u;  // f(0) = 0, f(1) = 1

// exclusive scan of 256 values in LDS (thread t gets the sum of 0..t-1)
template <typename T>
__device__ T wg_exclusive(T v, T *sh, T *total) {
  const uint32_t t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (uint32_t o = 1; o < DNA_THREADS; o <<= 1) {
    const T x = t >= o ? sh[t - o] : T(0);
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const T incl = sh[t];
  *total = sh[DNA_THREADS - 1];
  __syncthreads();
  return incl - v;
}

// run starts in a thread's DNA_PER elements
template <int E>
__device__ uint32_t run_starts(const void *buf, uint64_t n, uint32_t marker, uint64_t base, uint32_t *mask) {
  uint32_t prev = base > 0 && base - 1 < n ? elem_class<E>(buf, base - 1, marker) : DC_O;
  uint32_t m = 0;
  for (uint32_t k = 0; k < DNA_PER; k++) {
    const uint64_t i = base + k;
    const uint32_t c = i < n ? elem_class<E>(buf, i, marker) : DC_O;
    if (in_run(c) && !in_run(prev)) m |= 1u << k;
    prev = c;
  }
  *mask = m;
  return (uint32_t)__popcll((unsigned long long)m);
}

template <int E>
__global__ __launch_bounds__(DNA_THREADS) void k_dna_count(const void *buf, uint64_t n, uint32_t marker,
                                                           uint32_t *tile_cnt) {
  __shared__ uint32_t sh[DNA_THREADS];
  const uint64_t base = (uint64_t)blockIdx.x * DNA_TILE + (uint64_t)threadIdx.x * DNA_PER;
  uint32_t m;
  const uint32_t c = run_starts<E>(buf, n, marker, base, &m);
  uint32_t total;
  (void)wg_exclusive<uint32_t>(c, sh, &total);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = total;
}

// out[i] = in[0] + ... + in[i-1] for i <= m (one workgroup of 1024); with
// n_runs given, m is the number of groups of runs instead
__global__ __launch_bounds__(1024) void k_dna_scan(const uint32_t *in, uint64_t m, const uint64_t *n_runs,
                                                   uint64_t *out) {
  __shared__ uint64_t part[1024];
  const uint32_t t = threadIdx.x;
  if (n_runs) m = (*n_runs + DNA_THREADS - 1) / DNA_THREADS;
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < m; b0 += 1024) {
    const uint64_t j = b0 + t;
    const uint64_t v = j < m ? in[j] : 0;
    part[t] = v;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
      const uint64_t x = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += x;
      __syncthreads();
    }
    if (j < m) out[j] = carry + part[t] - v;
    carry += part[1023];
    __syncthreads();
  }
  if (t == 0) out[m] = carry;
}

template <int E>
__global__ __launch_bounds__(DNA_THREADS) void k_dna_runs(const void *buf, uint64_t n, uint32_t marker,
                                                          const uint64_t *tile_off, DnaRun *runs) {
  __shared__ uint32_t sh[DNA_THREADS];
  const uint64_t base = (uint64_t)blockIdx.x * DNA_TILE + (uint64_t)threadIdx.x * DNA_PER;
  uint32_t m;
  const uint32_t c = run_starts<E>(buf, n, marker, base, &m);
  uint32_t total;
  const uint32_t before = wg_exclusive<uint32_t>(c, sh, &total);
  uint64_t k = tile_off[blockIdx.x] + before;
  while (m) {
    const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    m &= m - 1u;
    runs[k++].a = base + b;
  }
}

// Walk one run; both matches and the map g.
template <int E>
__device__ void run_props(const void *buf, uint64_t n, uint32_t marker, DnaRun &R) {
  const uint64_t a = R.a;
  const uint32_t P = a > 0 ? elem_class<E>(buf, a - 1, marker) : DC_O;  // L or O
  const bool adj = P == DC_L && a >= 2 && in_run(elem_class<E>(buf, a - 2, marker));
  const bool starts_d = elem_class<E>(buf, a, marker) == DC_D;
  uint32_t prev = DC_O, cnt_u = 0;
  int64_t ld = -1, du = -1, ud = -1;  // last D; last D followed by U; first U followed by D
  uint32_t cu_ld = 0, cu_du = 0, cu_ud = 0;  // U's from a up to (and including) that element
  uint64_t i = a;
  for (; i < n; i++) {
    const uint32_t c = elem_class<E>(buf, i, marker);
    if (!in_run(c)) break;
    if (c == DC_U) {
      if (prev == DC_D) {
        du = (int64_t)(i - 1 - a);
        cu_du = cnt_u;
      }
      cnt_u++;
    } else {
      if (prev == DC_U && ud < 0) {
        ud = (int64_t)(i - 1 - a);
        cu_ud = cnt_u;
      }
      ld = (int64_t)(i - a);
      cu_ld = cnt_u;
    }
    prev = c;
  }
  const uint32_t S = i < n ? elem_class<E>(buf, i, marker) : DC_O;
  int64_t e = -1;  // last nucleotide of the match, from a
  uint32_t ue = 0;  // U's from a to e
  bool consumes = false;
  if (prev == DC_D && S == DC_L) {
    e = (int64_t)(i - 1 - a);
    ue = cnt_u;
    consumes = true;
  } else if (prev == DC_U) {
    e = ld;
    ue = cu_ld;
  } else {
    e = du;
    ue = cu_du;
  }
  uint32_t f = adj ? DR_ADJ : 0u;
  if (e >= 0 && starts_d && P == DC_L) {
    f |= DR_A;
    R.lenA = (uint32_t)(e + 1);
    R.nuA = ue;
  }
  if (e >= 0 && ud >= 0 && ud + 1 <= e) {
    f |= DR_B;
    R.offB = (uint32_t)(ud + 1);
    R.lenB = (uint32_t)(e - ud);
    R.nuB = ue - cu_ud;
  }
  if (consumes) {
    f |= DR_CONSUMES;
    // consumed when a match is made: A needs the newline before the run to
    // be free (not consumed by the previous run when adjacent)
    const bool m0 = (f & DR_A) || (f & DR_B);
    const bool m1 = ((f & DR_A) && !adj) || (f & DR_B);
    f |= (m0 ? DR_G0 : 0u) | (m1 ? DR_G1 : 0u);
  }
  R.flags = f;
}

__device__ __forceinline__ uint32_t run_map(uint32_t flags) {
  return ((flags & DR_G0) ? 1u : 0u) | ((flags & DR_G1) ? 2u : 0u);
}

// composition of maps over a workgroup (thread t gets map_0 then .. then map_{t-1})
__device__ uint32_t wg_map_exclusive(uint32_t g, uint32_t *sh, uint32_t *total) {
  const uint32_t t = threadIdx.x;
  sh[t] = g;
  __syncthreads();
  for (uint32_t o = 1; o < DNA_THREADS; o <<= 1) {
    const uint32_t x = t >= o ? sh[t - o] : MAP_ID;
    __syncthreads();
    sh[t] = map_then(x, sh[t]);
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[DNA_THREADS - 1];
  const uint32_t excl = t > 0 ? sh[t - 1] : MAP_ID;
  __syncthreads();
  (void)incl;
  return excl;
}

template <int E>
__global__ __launch_bounds__(DNA_THREADS) void k_dna_props(const void *buf, uint64_t n, uint32_t marker,
                                                           const uint64_t *n_runs, DnaRun *runs, uint32_t *grp_map) {
  __shared__ uint32_t sh[DNA_THREADS];
  const uint64_t R = *n_runs;
  for (uint64_t g0 = (uint64_t)blockIdx.x * DNA_THREADS; g0 < R; g0 += (uint64_t)gridDim.x * DNA_THREADS) {
    const uint64_t k = g0 + threadIdx.x;
    uint32_t g = MAP_ID;
    if (k < R) {
      DnaRun r = runs[k];
      run_props<E>(buf, n, marker, r);
      runs[k] = r;
      g = run_map(r.flags);
    }
    uint32_t total;
    (void)wg_map_exclusive(g, sh, &total);
    if (threadIdx.x == 0) grp_map[g0 / DNA_THREADS] = total;
  }
}

// bit entering each group: the composed maps of the groups before it,
// applied to 0 (nothing precedes the first run)
__global__ __launch_bounds__(1024) void k_dna_chain(const uint32_t *grp_map, const uint64_t *n_runs,
                                                    uint32_t *grp_in) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint64_t G = (*n_runs + DNA_THREADS - 1) / DNA_THREADS;
  uint32_t carry = MAP_ID;
  for (uint64_t b0 = 0; b0 < G; b0 += 1024) {
    const uint64_t j = b0 + t;
    const uint32_t v = j < G ? grp_map[j] : MAP_ID;
    part[t] = v;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
      const uint32_t x = t >= o ? part[t - o] : MAP_ID;
      __syncthreads();
      part[t] = map_then(x, part[t]);
      __syncthreads();
    }
    const uint32_t excl = map_then(carry, t > 0 ? part[t - 1] : MAP_ID);
    if (j < G) grp_in[j] = excl & 1u;  // the composed map at 0
    carry = map_then(carry, part[1023]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(DNA_THREADS) void k_dna_select(const uint64_t *n_runs, DnaRun *runs,
                                                            const uint32_t *grp_in, uint32_t min_len,
                                                            uint32_t *grp_cnt) {
  __shared__ uint32_t sh[DNA_THREADS];
  const uint64_t R = *n_runs;
  for (uint64_t g0 = (uint64_t)blockIdx.x * DNA_THREADS; g0 < R; g0 += (uint64_t)gridDim.x * DNA_THREADS) {
    const uint64_t k = g0 + threadIdx.x;
    uint32_t flags = k < R ? runs[k].flags : 0u;
    uint32_t total;
    const uint32_t pre = wg_map_exclusive(k < R ? run_map(flags) : MAP_ID, sh, &total);
    const uint32_t cin = (pre >> grp_in[g0 / DNA_THREADS]) & 1u;  // previous run consumed the newline
    uint32_t acc = 0;
    if (k < R) {
      const DnaRun r = runs[k];
      uint32_t len = 0;
      if ((flags & DR_A) && !((flags & DR_ADJ) && cin)) {
        flags |= DR_TAKE_A;
        len = r.lenA;
      } else if (flags & DR_B) {
        flags |= DR_TAKE_B;
        len = r.lenB;
      }
      if ((flags & (DR_TAKE_A | DR_TAKE_B)) && len >= min_len) {
        flags |= DR_ACCEPT;
        acc = 1;
      }
      runs[k].flags = flags;
    }
    uint32_t cnt;
    (void)wg_exclusive<uint32_t>(acc, sh, &cnt);
    if (threadIdx.x == 0) grp_cnt[g0 / DNA_THREADS] = cnt;
  }
}

__global__ __launch_bounds__(DNA_THREADS) void k_dna_write(const uint64_t *n_runs, const DnaRun *runs,
                                                           const uint64_t *grp_off, gz_dna_seq *seqs,
                                                           uint64_t max_seqs, const uint64_t *bounds,
                                                           uint32_t n_ranges, uint32_t *stats) {
  __shared__ uint32_t sh[DNA_THREADS];
  const uint64_t R = *n_runs;
  for (uint64_t g0 = (uint64_t)blockIdx.x * DNA_THREADS; g0 < R; g0 += (uint64_t)gridDim.x * DNA_THREADS) {
    const uint64_t k = g0 + threadIdx.x;
    const DnaRun r = k < R ? runs[k] : DnaRun{};
    const uint32_t acc = (k < R && (r.flags & DR_ACCEPT)) ? 1u : 0u;
    uint32_t cnt;
    const uint32_t rank = wg_exclusive<uint32_t>(acc, sh, &cnt);
    if (acc) {
      gz_dna_seq s;
      const bool A = (r.flags & DR_TAKE_A) != 0;
      s.start = r.a + (A ? 0u : r.offB);
      s.len = A ? r.lenA : r.lenB;
      s.n_undetermined = A ? r.nuA : r.nuB;
      const uint64_t o = grp_off[g0 / DNA_THREADS] + rank;
      if (o < max_seqs) seqs[o] = s;
      if (n_ranges && s.start >= bounds[0] && s.start < bounds[n_ranges]) {
        // the last range whose first position is at or before the start
        uint32_t lo = 0, hi = n_ranges;
        for (int it = 0; it < 40 && hi - lo > 1; it++) {
          const uint32_t mid = (lo + hi) >> 1;
          if (bounds[mid] <= s.start) lo = mid;
          else hi = mid;
        }
        atomicAdd(&stats[3u * lo], 1u);
        if (s.n_undetermined) atomicAdd(&stats[3u * lo + 1u], 1u);
      }
    }
  }
}

__global__ __launch_bounds__(DNA_THREADS) void k_dna_zero(uint32_t *stats, uint32_t n) {
  for (uint32_t i = blockIdx.x * DNA_THREADS + threadIdx.x; i < n; i += gridDim.x * DNA_THREADS) stats[i] = 0;
}

__global__ __launch_bounds__(DNA_THREADS) void k_dna_resolve(uint32_t *stats, uint32_t n_ranges, uint32_t threshold,
                                                             const uint64_t *grp_off, const uint64_t *n_runs,
                                                             uint64_t *n_seqs) {
  for (uint32_t r = blockIdx.x * DNA_THREADS + threadIdx.x; r < n_ranges; r += gridDim.x * DNA_THREADS)
    stats[3u * r + 2u] = (stats[3u * r] >= threshold && stats[3u * r + 1u] == 0) ? 1u : 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_seqs = grp_off[(*n_runs + DNA_THREADS - 1) / DNA_THREADS];
}

}  // namespace gzgpu

using namespace gzgpu;

// Workspace of gzk_dna for n elements; pieces in order, 256-byte aligned.
struct DnaLayout {
  uint64_t tile_cnt, tile_off, runs, grp_map, grp_in, grp_cnt, grp_off, total;
  uint64_t tiles, max_runs, groups;
};

static uint64_t dna_align(uint64_t x) { return (x + 255u) & ~255ull; }

static DnaLayout dna_layout(uint64_t n) {
  DnaLayout L{};
  L.tiles = (n + DNA_TILE - 1) / DNA_TILE;
  L.max_runs = (n + 1) / 2;
  L.groups = (L.max_runs + DNA_THREADS - 1) / DNA_THREADS;
  uint64_t o = 0;
  L.tile_cnt = o; o = dna_align(o + 4 * (L.tiles + 1));
  L.tile_off = o; o = dna_align(o + 8 * (L.tiles + 1));
  L.runs = o; o = dna_align(o + sizeof(DnaRun) * L.max_runs);
  L.grp_map = o; o = dna_align(o + 4 * (L.groups + 1));
  L.grp_in = o; o = dna_align(o + 4 * (L.groups + 1));
  L.grp_cnt = o; o = dna_align(o + 4 * (L.groups + 1));
  L.grp_off = o; o = dna_align(o + 8 * (L.groups + 1));
  L.total = o;
  return L;
}

extern "C" {

uint64_t gzk_dna_ws(uint64_t n) { return dna_layout(n).total; }

hipError_t gzk_dna(const void *buf, uint64_t n, uint32_t elem_bytes, uint32_t marker, uint32_t min_len,
                   gz_dna_seq *seqs, uint64_t max_seqs, uint64_t *n_seqs, const uint64_t *bounds, uint32_t n_ranges,
                   uint32_t threshold, uint32_t *stats, uint8_t *ws, hipStream_t st) {
  const DnaLayout L = dna_layout(n);
  uint32_t *tile_cnt = (uint32_t *)(ws + L.tile_cnt);
  uint64_t *tile_off = (uint64_t *)(ws + L.tile_off);
  DnaRun *runs = (DnaRun *)(ws + L.runs);
  uint32_t *grp_map = (uint32_t *)(ws + L.grp_map);
  uint32_t *grp_in = (uint32_t *)(ws + L.grp_in);
  uint32_t *grp_cnt = (uint32_t *)(ws + L.grp_cnt);
  uint64_t *grp_off = (uint64_t *)(ws + L.grp_off);
  const uint64_t *n_runs = tile_off + L.tiles;
  const uint32_t T = (uint32_t)L.tiles;
  // persistent grids for the per-run passes
  const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(L.groups, 1), 8192);
  if (n_ranges) hipLaunchKernelGGL(k_dna_zero, dim3(std::min<uint32_t>((3 * n_ranges + 255) / 256, 1024)),
                                   dim3(DNA_THREADS), 0, st, stats, 3 * n_ranges);
  if (T) {
    if (elem_bytes == 2) hipLaunchKernelGGL(k_dna_count<2>, dim3(T), dim3(DNA_THREADS), 0, st, buf, n, marker, tile_cnt);
    else hipLaunchKernelGGL(k_dna_count<1>, dim3(T), dim3(DNA_THREADS), 0, st, buf, n, marker, tile_cnt);
  }
  hipLaunchKernelGGL(k_dna_scan, dim3(1), dim3(1024), 0, st, tile_cnt, L.tiles, (const uint64_t *)nullptr, tile_off);
  if (T) {
    if (elem_bytes == 2) hipLaunchKernelGGL(k_dna_runs<2>, dim3(T), dim3(DNA_THREADS), 0, st, buf, n, marker, tile_off, runs);
    else hipLaunchKernelGGL(k_dna_runs<1>, dim3(T), dim3(DNA_THREADS), 0, st, buf, n, marker, tile_off, runs);
  }
  if (elem_bytes == 2)
    hipLaunchKernelGGL(k_dna_props<2>, dim3(grid), dim3(DNA_THREADS), 0, st, buf, n, marker, n_runs, runs, grp_map);
  else
    hipLaunchKernelGGL(k_dna_props<1>, dim3(grid), dim3(DNA_THREADS), 0, st, buf, n, marker, n_runs, runs, grp_map);
  hipLaunchKernelGGL(k_dna_chain, dim3(1), dim3(1024), 0, st, grp_map, n_runs, grp_in);
  hipLaunchKernelGGL(k_dna_select, dim3(grid), dim3(DNA_THREADS), 0, st, n_runs, runs, grp_in, min_len, grp_cnt);
  hipLaunchKernelGGL(k_dna_scan, dim3(1), dim3(1024), 0, st, grp_cnt, L.groups, n_runs, grp_off);
  hipLaunchKernelGGL(k_dna_write, dim3(grid), dim3(DNA_THREADS), 0, st, n_runs, runs, grp_off, seqs, max_seqs,
                     bounds, n_ranges, stats);
  hipLaunchKernelGGL(k_dna_resolve, dim3(std::min<uint32_t>((n_ranges + 255) / 256 + 1, 1024)), dim3(DNA_THREADS), 0,
                     st, stats, n_ranges, threshold, grp_off, n_runs, n_seqs);
  return hipGetLastError();
}

}  // extern "C"
