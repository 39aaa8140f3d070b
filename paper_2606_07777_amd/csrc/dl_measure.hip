// Measurement helper: the sustained HBM read rate of this device, taken with a
// plain streaming kernel (no arithmetic beyond folding the loaded words), as
// the practical ceiling the memory-bound gradient pass is compared against.
#include "dl_common.h"

namespace {

typedef unsigned dl_v4u __attribute__((ext_vector_type(4)));

// Grid-stride read of n16 16-byte words with the nontemporal hint (the data is
// streamed once); each thread keeps four loads in flight per step and folds
// them with XOR so none can be elided.  One word per workgroup reaches memory
// (XOR-folded into *sink).  Of the shapes measured (loads in flight per
// thread, contiguous or strided blocks, 4 to 64 workgroups per compute unit,
// with and without the hint), this one read fastest.
__global__ void __launch_bounds__(256) stream_read(const dl_v4u* __restrict__ src, int64_t n16,
                                                   unsigned* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  dl_v4u acc = {0u, 0u, 0u, 0u};
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const dl_v4u a = __builtin_nontemporal_load(src + i);
    const dl_v4u b = __builtin_nontemporal_load(src + i + stride);
    const dl_v4u c = __builtin_nontemporal_load(src + i + 2 * stride);
    const dl_v4u d = __builtin_nontemporal_load(src + i + 3 * stride);
    acc ^= a ^ b ^ c ^ d;
  }
  for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(src + i);
  unsigned v = acc.x ^ acc.y ^ acc.z ^ acc.w;
  for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
  __shared__ unsigned sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) atomicXor(sink, sh[0] ^ sh[1] ^ sh[2] ^ sh[3]);
}

}  // namespace

extern "C" dl_status dl_read_bandwidth(int64_t bytes, int32_t reps, void* stream, double* gbps) {
  DL_CHECK_ARG(gbps && bytes >= 16 && reps >= 1, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, n_cu = 0;
  DL_HIP_TRY(hipGetDevice(&dev));
  DL_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n16 = bytes / 16;
  // a buffer of its own (hipMalloc), so the figure does not depend on how a
  // caller's allocator laid its memory out; one extra word for the sink
  unsigned char* buf = nullptr;
  DL_HIP_TRY(hipMalloc((void**)&buf, (size_t)n16 * 16 + 256));
  struct Free {
    void* p;
    ~Free() { (void)hipFree(p); }
  } guard{buf};
  unsigned* sink = reinterpret_cast<unsigned*>(buf + (size_t)n16 * 16);
  DL_HIP_TRY(hipMemsetAsync(buf, 1, (size_t)n16 * 16 + 256, st));
  const unsigned grid = (unsigned)std::max(1, n_cu * 64);
  // one untimed launch brings the kernel and the clocks up
  hipLaunchKernelGGL(stream_read, dim3(grid), dim3(256), 0, st, (const dl_v4u*)buf, n16, sink);
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
    hipLaunchKernelGGL(stream_read, dim3(grid), dim3(256), 0, st, (const dl_v4u*)buf, n16, sink);
    if (hipGetLastError() != hipSuccess) rc = DL_EHIP;
  }
  float ms = 0.f;
  if (rc == DL_OK && hipEventRecord(e1, st) != hipSuccess) rc = DL_EHIP;
  if (rc == DL_OK && hipEventSynchronize(e1) != hipSuccess) rc = DL_EHIP;
  if (rc == DL_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DL_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == DL_OK && hipStreamSynchronize(st) != hipSuccess) rc = DL_EHIP;
  if (rc != DL_OK) {
    dl_set_error("timing the read kernel failed");
    return rc;
  }
  *gbps = (double)(n16 * 16) * reps / (ms * 1e-3) / 1e9;
  return DL_OK;
}
