// Internal launcher interface between the C-ABI layer (api.cpp) and the
// kernel translation units.  Launchers assume validated arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pauli {

enum Dir { FORWARD = 0, ADJOINT = 1 };

// Binary64 Gray-code kernel.  FORWARD: in = G (matrix), out = coefficients;
// ADJOINT: in = coefficients, out = matrix.  scale multiplies the result
// (2^-N forward and for the gradient, 1 for recomposition).
hipError_t launch_gray(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N,
                       int batch, double scale, hipStream_t stream);

// Matrix-core contraction.  planes = 3 (split bf16) or 1 (fp32).
// tile = 1-based tile id (0 = default for N).  ws = device scratch of
// mfma_workspace_bytes(planes, N, batch) bytes for the packed operand.
hipError_t launch_mfma(Dir dir, int planes, const void* in, bool in_c128, void* out,
                       bool out_c128, int N, int batch, double scale, int tile, void* ws,
                       hipStream_t stream);
size_t mfma_workspace_bytes(int planes, int N, int batch);
int mfma_tile_count(int planes);
bool mfma_tile_valid(int planes, int tile, int N);
int mfma_default_tile(int planes, int N);

// Uneven batch: device descriptor table built by the host.
struct BatchItem {
    const void* in;   // matrix of order 2^n
    void* out;        // 4^n coefficients
    int n;            // qubit count
    int tile0;        // first linear tile id of this matrix in the work list
};
size_t batched_workspace_bytes(int count);
hipError_t launch_batched(int planes, const BatchItem* items_dev, int count, int total_tiles,
                          unsigned int* counter_dev, hipStream_t stream);
int batched_tiles_for(int n);

}  // namespace pauli
