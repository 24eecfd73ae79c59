// Test-only: the block-start table check of the scan (check_dynamic_tables)
// against the table reader of the decoder (read_dynamic_tables, strict,
// nothing stored) at given candidate bits, in the CPU executor.  This file
// is the executor's translation unit for the kernels: it includes their
// source, then adds the comparison kernel.
#include "gz_kernels.hip"

using namespace gzgpu;

namespace {

__global__ void k_stage2_diff(const uint8_t *buf, uint64_t n, const uint64_t *bits, int nb, int32_t *res_read,
                              int32_t *res_check) {
  __shared__ TablesLDS sh;
  Src s;
  s.init(buf, n);
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
                               int32_t *res_check) {
  hipLaunchKernelGGL(k_stage2_diff, dim3(1), dim3(64), 0, 0, buf, n, bits, nb, res_read, res_check);
  return 0;
}
