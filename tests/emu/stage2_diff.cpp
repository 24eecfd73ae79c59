// Test-only: the block-start table checks of the scan (check_dynamic_tables,
// whole wave; lane_tables_ok, one candidate per lane) against the table
// reader of the decoder (read_dynamic_tables, strict, nothing stored) at
// given candidate bits, in the CPU executor.  This file
// is the executor's translation unit for the kernels: it includes their
// source, then adds the comparison kernel.
#include "gz_kernels.hip"

using namespace gzgpu;

namespace {

__global__ void k_stage2_diff(const uint8_t *buf, uint64_t n, const uint64_t *bits, int nb, int32_t *res_read,
                              int32_t *res_check, int32_t *res_lane) {
  __shared__ TablesLDS sh;
  __shared__ uint8_t tab[128 * 64];
  Src s;
  s.init(buf, n);
  // one candidate per lane
  for (int i0 = 0; i0 < nb; i0 += 64) {
    const int i = i0 + (int)threadIdx.x;
    if (i < nb) res_lane[i] = lane_tables_ok(s, bits[i], tab, (int)threadIdx.x, 0u) ? 1 : 0;
  }
  for (int i = 0; i < nb; i++) {
    WaveBits a;
    a.s = s;
    a.init(bits[i] + 3);
    bool nd;
    const int r0 = read_dynamic_tables(a, sh, true, false, &nd);
    WaveBits b;
    b.s = s;
    b.init(bits[i] + 3);
    const int r1 = check_dynamic_tables(b, sh);
    if (threadIdx.x == 0) {
      res_read[i] = r0 == D_OK ? 1 : 0;
      res_check[i] = r1 == D_OK ? 1 : 0;
    }
  }
}

}  // namespace

extern "C" int emu_stage2_diff(const uint8_t *buf, uint64_t n, const uint64_t *bits, int nb, int32_t *res_read,
                               int32_t *res_check, int32_t *res_lane) {
  hipLaunchKernelGGL(k_stage2_diff, dim3(1), dim3(64), 0, 0, buf, n, bits, nb, res_read, res_check, res_lane);
  return 0;
}
