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

// Matrix-core contraction.  planes = 3 (split bf16), 2 (split fp16) or 1 (fp32).
// tile = 1-based tile id (0 = default for N).  ws = device scratch of
// mfma_workspace_bytes(planes, N, batch) bytes for the packed operand.
hipError_t launch_mfma(Dir dir, int planes, const void* in, bool in_c128, void* out,
                       bool out_c128, int N, int batch, double scale, int tile, void* ws,
                       hipStream_t stream);
size_t mfma_workspace_bytes(int planes, int N, int batch);
hipError_t launch_mfma_pack(Dir dir, int planes, const void* in, bool in_c128, int N, int batch, void* ws,
                            hipStream_t stream);
hipError_t launch_mfma_contract(Dir dir, int planes, const void* ws, void* out, bool out_c128, int N, int batch,
                                double scale, int tile, hipStream_t stream);
// Hermitian input, forward only: half of K for most flip-mask tiles and
// exactly real coefficients; register-ring tiles only.
hipError_t launch_mfma_hermitian(int planes, const void* in, bool in_c128, void* out, bool out_c128, int N,
                                 int batch, double scale, int tile, void* ws, hipStream_t stream);
hipError_t launch_mfma_pack_hermitian(int planes, const void* in, bool in_c128, int N, int batch, void* ws,
                                      hipStream_t stream);
hipError_t launch_mfma_contract_hermitian(int planes, const void* ws, void* out, bool out_c128, int N, int batch,
                                          double scale, int tile, hipStream_t stream);
bool mfma_tile_valid_hermitian(int planes, int tile, int N);
int mfma_default_tile_hermitian(int planes, int N);
int mfma_tile_count(int planes);
bool mfma_tile_valid(int planes, int tile, int N);
int mfma_default_tile(int planes, int N);

// Fixed-point int8 contraction: the input (G, or the coefficients for
// ADJOINT) quantised per matrix to integers of at most 23 bits, split into
// three int8 digit planes, summed exactly by int8 MFMA.  ws = device scratch
// of i8_workspace_bytes(N, batch).  herm (FORWARD only): Hermitian G (half of
// K and of the rows for most flip masks; the same result bit for bit).
size_t i8_workspace_bytes(int N, int batch);
hipError_t launch_i8(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N, int batch, double scale,
                     void* ws, bool herm, hipStream_t stream);
// The two halves of launch_i8: scale + quantise + pack, then the contraction.
hipError_t launch_i8_pack(const void* in, bool in_c128, int N, int batch, void* ws, Dir dir, bool herm,
                          hipStream_t stream);
hipError_t launch_i8_contract(const void* ws, void* out, bool out_c128, int N, int batch, double scale, Dir dir,
                              bool herm, hipStream_t stream);

// Uneven batch: device descriptor table built by the host, one entry per
// matrix in processing order.
struct BatchItem {
    const void* in;   // complex64 matrix of order 2^n
    void* out;        // its 4^n complex64 coefficients
    size_t ws_off;    // byte offset of its packed operand in the packed area
    int n;            // qubit count
    uint32_t pack0;   // first pack tile of this matrix in the batch numbering
    uint32_t tile0;   // first output tile of this matrix in the batch numbering
};
int batched_tile_count();
bool batched_tile_valid(int planes, int btile);
int batched_default_tile(int planes);
uint32_t batched_output_tiles(int btile, int n);
uint32_t batched_pack_tiles(int n);
size_t batched_packed_bytes(int planes, int n);
// pack_slot_dev[t] / tile_slot_dev[t] = descriptor slot of the matrix owning
// pack tile t / output tile t.  queues_dev = [nq | nq + 1 offsets | output
// tile ids] with 1 <= nq <= MAX_QUEUES and nq <= tile_total: queue q's tiles
// are claimed, through counter_dev[q], by the workgroups whose index is q
// modulo nq.  The pack launch also zeroes counter_dev[0 .. MAX_QUEUES).
// planes = 2 also needs pe_dev (count ints: each slot's prescale exponent)
// and partial_dev (pack_total floats), both written before they are read.
constexpr uint32_t MAX_QUEUES = 8;   // one per XCD
hipError_t launch_batched(int planes, int btile, const BatchItem* items_dev, const uint32_t* pack_slot_dev,
                          const uint32_t* tile_slot_dev, const uint32_t* queues_dev, uint32_t count,
                          uint32_t pack_total, uint32_t tile_total, unsigned char* packed, unsigned int* counter_dev,
                          int* pe_dev, float* partial_dev, hipStream_t stream);

// Pauli-string list: the host sorts the strings into chunks of at most 256
// strings sharing a line group (flip masks equal above bit 3); chunk k covers
// entries[first, first + count) and the masks x0 .. x0 + 15 (x0 = 0 for N < 4).
struct StringChunk {
    uint32_t x0, first, count, pad;
};
struct StringEntry {
    uint32_t n;      // Pauli string index (< 4^N)
    uint32_t slot;   // position of its coefficient in the output
};
constexpr int STRINGS_PER_CHUNK = 256;
constexpr int STRINGS_MAX_BLOCKS = 2048;   // chunks x parts aimed for when the list is short
// Column batches of one line-group pass at order N (the most parts a chunk can split into).
uint32_t strings_batches(int N);
// parts > 1 splits every chunk's columns over `parts` workgroups whose binary64
// partial sums (parts x count double2 in `partial`, indexed by entry) are then
// added in order by a second kernel.
hipError_t launch_strings(const void* G, bool in_c128, int N, const StringChunk* chunks, int nchunks,
                          const StringEntry* entries, int count, int parts, double2* partial, void* out,
                          bool out_c128, hipStream_t stream);
// Adjoint of the list (dense 2^N x 2^N output): entries sorted by flip mask,
// first[x] .. first[x + 1] (2^N + 1 offsets) the strings of mask x.
hipError_t launch_strings_adjoint(const void* grad, bool grad_c128, const StringEntry* entries,
                                  const uint32_t* first, void* out, bool out_c128, int N, hipStream_t stream);

// All coefficients by two fast Walsh-Hadamard passes through an intermediate
// of fwht_workspace_bytes(N, batch, narrow) bytes: binary64 pairs (16 bytes
// per element), or binary32 pairs (8 bytes) when narrow.
constexpr int FWHT_N_MIN = 0, FWHT_N_MAX = 16;
constexpr int FWHT_SMALL_N_MAX = 8;   // up to here one kernel works in LDS and needs no workspace
bool fwht_supported(int N);
size_t fwht_workspace_bytes(int N, int batch, bool narrow);
// FORWARD: in = matrices, out = coefficients; ADJOINT: in = coefficients,
// out = matrices.  scale multiplies the result as for launch_gray.
hipError_t launch_fwht(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N, int batch,
                       double scale, bool narrow, void* ws, hipStream_t stream);

}  // namespace pauli
