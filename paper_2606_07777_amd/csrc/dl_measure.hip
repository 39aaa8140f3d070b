// Measurement helper: the sustained HBM read rate of this device, taken with a
// plain streaming kernel (no arithmetic beyond folding the loaded words), as
// the practical ceiling the memory-bound gradient pass is compared against.
#include "dl_common.h"

namespace {

// Grid-stride read of n16 16-byte words; each thread keeps four loads in
// flight per step and folds them with XOR so none can be elided.  One word per
// workgroup reaches memory (XOR-folded into *sink).
__global__ void __launch_bounds__(256) stream_read(const uint4* __restrict__ src, int64_t n16,
                                                   unsigned* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc.x ^= a.x ^ b.x ^ c.x ^ d.x;
    acc.y ^= a.y ^ b.y ^ c.y ^ d.y;
    acc.z ^= a.z ^ b.z ^ c.z ^ d.z;
    acc.w ^= a.w ^ b.w ^ c.w ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 a = src[i];
    acc.x ^= a.x;
    acc.y ^= a.y;
    acc.z ^= a.z;
    acc.w ^= a.w;
  }
  unsigned v = acc.x ^ acc.y ^ acc.z ^ acc.w;
  for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
  __shared__ unsigned sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicXor(sink, sh[0] ^ sh[1] ^ sh[2] ^ sh[3]);
}

}  // namespace

extern "C" dl_status dl_read_bandwidth(const void* buf, int64_t bytes, int32_t reps, void* stream, unsigned* sink,
                                       double* gbps) {
  DL_CHECK_ARG(buf && sink && gbps && bytes >= 16 && reps >= 1, "bad argument");
  DL_CHECK_ARG(((uintptr_t)buf & 15) == 0, "buf must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, n_cu = 0;
  DL_HIP_TRY(hipGetDevice(&dev));
  DL_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n16 = bytes / 16;
  const unsigned grid = (unsigned)std::max(1, n_cu * 16);
  // one untimed launch brings the kernel and the clocks up
  hipLaunchKernelGGL(stream_read, dim3(grid), dim3(256), 0, st, (const uint4*)buf, n16, sink);
  DL_HIP_TRY(hipGetLastError());
  hipEvent_t e0, e1;
  DL_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    dl_set_error("hipEventCreate failed");
    return DL_EHIP;
  }
  dl_status rc = DL_OK;
  if (hipEventRecord(e0, st) != hipSuccess) rc = DL_EHIP;
  for (int r = 0; r < reps && rc == DL_OK; ++r) {
    hipLaunchKernelGGL(stream_read, dim3(grid), dim3(256), 0, st, (const uint4*)buf, n16, sink);
    if (hipGetLastError() != hipSuccess) rc = DL_EHIP;
  }
  float ms = 0.f;
  if (rc == DL_OK && hipEventRecord(e1, st) != hipSuccess) rc = DL_EHIP;
  if (rc == DL_OK && hipEventSynchronize(e1) != hipSuccess) rc = DL_EHIP;
  if (rc == DL_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DL_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DL_OK) {
    dl_set_error("timing the read kernel failed");
    return rc;
  }
  *gbps = (double)(n16 * 16) * reps / (ms * 1e-3) / 1e9;
  return DL_OK;
}
