// Uneven batch (placeholder until the persistent kernel lands).
#include "common.hpp"
#include "internal.hpp"

namespace pauli {
size_t batched_workspace_bytes(int count) { return ((sizeof(BatchItem) * count + 255) / 256) * 256 + 256; }
int batched_tiles_for(int n) { return 1 << (n > 5 ? n - 5 : 0); }
hipError_t launch_batched(int, const BatchItem*, int, int, unsigned int*, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace pauli
