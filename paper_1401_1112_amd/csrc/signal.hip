// Scalar records to the host with a completion word.
#include "signal.h"

namespace amrfld {

namespace {

constexpr int kSignalThreads = 256;

__global__ __launch_bounds__(kSignalThreads) void k_scalars_to_host(const uint64_t* __restrict__ src,
                                                                    uint64_t* __restrict__ dst, int n_words,
                                                                    uint64_t* seq, uint64_t value) {
  for (int i = int(threadIdx.x); i < n_words; i += kSignalThreads) dst[i] = src[i];
  __threadfence_system();  // this thread's words reach host memory before anything it stores later
  __syncthreads();         // every thread has passed its fence
  if (threadIdx.x == 0) __hip_atomic_store(seq, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

void launch_scalars_to_host(hipStream_t s, const void* src, void* dst, int n_words, uint64_t* seq,
                            uint64_t value) {
  hipLaunchKernelGGL(k_scalars_to_host, dim3(1), dim3(kSignalThreads), 0, s,
                     static_cast<const uint64_t*>(src), static_cast<uint64_t*>(dst), n_words, seq, value);
}

}  // namespace amrfld
