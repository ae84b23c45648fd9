// Scalar records to the host with a completion word: the host waits by reading
// pinned memory instead of synchronising the stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amrfld {

// Copies n_words 8-byte words from device memory to the device-mapped view of
// pinned, coherent host memory, then stores `value` to *seq (also mapped host
// memory) once every copied word is visible to the host.  One block.
void launch_scalars_to_host(hipStream_t s, const void* src, void* dst, int n_words, uint64_t* seq,
                            uint64_t value);

}  // namespace amrfld
