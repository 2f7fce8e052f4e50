// Uneven batch: many matrices of different order decomposed by one batched
// pack launch and one persistent contraction launch (the paper's embarrassing
// parallelism over coefficients, section 3, extended over matrices).
//
// The host builds a descriptor table in device memory: one entry per matrix,
// in decreasing order of N (longest-processing-time first), with the matrix's
// packed-operand offset and its first pack tile and first output tile in the
// batch-wide numbering, followed by the slot of every pack tile and of every
// output tile.  A pack workgroup finds its matrix with one read of the pack
// slot table.  The contraction kernel is persistent: each workgroup takes
// output tiles from a single atomic counter until the list is exhausted, so
// every workgroup ends once the counter passes the last tile and the grid
// drains.  It claims its next tile when it starts the current one (the
// atomic's round trip then overlaps the contraction) and finds a tile's
// matrix with one read of the output slot table.  The pack kernel's first
// thread zeroes the counter: the contraction runs after the pack on the same
// stream, and the previous contraction has finished before the pack starts
// (no memset node, so the sequence can be captured in a HIP graph and
// replayed).  The two-plane split first finds every matrix's prescale: one
// reduction workgroup per pack tile takes the largest component of an equal
// share of its matrix, then one workgroup per matrix reduces its shares.
#include "mfma_tile.hpp"

namespace pauli {
namespace {

using namespace mfma;

// Share t of its matrix (pack tile t): 4^n / pack_tiles(n) consecutive
// elements, an integer count (32 x 128 for n >= 7, the whole matrix below 5).
__global__ __launch_bounds__(256) void absmax_batched_kernel(const BatchItem* __restrict__ items,
                                                             const uint32_t* __restrict__ pack_slot,
                                                             float* __restrict__ partial) {
    __shared__ float red[4];
    const BatchItem it = items[pack_slot[blockIdx.x]];
    const size_t n = (size_t)1 << (2 * it.n);
    const size_t per = n / pack_tiles(it.n);
    const float2* p = (const float2*)it.in + (size_t)(blockIdx.x - it.pack0) * per;
    float m = 0.f;
    for (size_t i = threadIdx.x; i < per; i += 256) {
        const float2 v = p[i];
        m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf(v.x), __builtin_fabsf(v.y)));
    }
    m = block_max256(m, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// One workgroup per descriptor slot: the matrix's prescale exponent.
__global__ __launch_bounds__(256) void prescale_batched_kernel(const BatchItem* __restrict__ items,
                                                               const float* __restrict__ partial,
                                                               int* __restrict__ pe) {
    __shared__ float red[4];
    const BatchItem it = items[blockIdx.x];
    const uint32_t tiles = pack_tiles(it.n);
    float m = 0.f;
    for (uint32_t i = threadIdx.x; i < tiles; i += 256) m = __builtin_fmaxf(m, partial[it.pack0 + i]);
    m = block_max256(m, red);
    if (threadIdx.x == 0) pe[blockIdx.x] = prescale_exponent(m);
}

template <int PLANES>
__global__ __launch_bounds__(256) void pack_batched_kernel(const BatchItem* __restrict__ items,
                                                           const uint32_t* __restrict__ pack_slot,
                                                           unsigned char* __restrict__ ws,
                                                           unsigned int* __restrict__ counter,
                                                           const int* __restrict__ pe) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[pack_lds_bytes<PLANES>()];
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;   // for the contraction that follows
    const uint32_t slot = pack_slot[blockIdx.x];
    const BatchItem it = items[slot];
    pack_tile<PLANES, FORWARD, false>((const unsigned char*)it.in, ws + it.ws_off, it.n,
                                      blockIdx.x - it.pack0, lds, PLANES == 2 ? pe[slot] : 0);
}

// AHEAD > 0: output tiles of matrices with at least MT rows and a whole
// number of sign groups of slice pairs take the LDS-staged contraction
// (each fragment copied once per workgroup, AHEAD pairs ahead); smaller ones
// take the register ring.
template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0>
__device__ __attribute__((always_inline)) inline void batched_loop(const BatchItem* __restrict__ items,
                                                                   const uint32_t* __restrict__ tile_slot,
                                                                   uint32_t total, const unsigned char* __restrict__ ws,
                                                                   unsigned int* __restrict__ counter,
                                                                   const int* __restrict__ pe,
                                                                   unsigned char* lds, uint32_t& next) {
    static_assert(AHEAD == 0 || WAVES == 4, "the LDS-staged contraction runs four waves per workgroup");
    constexpr int MT = WAVES * RB * 32;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t t = next;
    __syncthreads();                   // everyone has read `next` before it is rewritten
    while (t < total) {                // uniform: every workgroup leaves once the list is done
        uint32_t claimed = 0;
        if (threadIdx.x == 0) claimed = atomicAdd(counter, 1u);   // read only after this tile
        const uint32_t slot = tile_slot[t];
        const BatchItem it = items[slot];
        const uint32_t Dp = padded_dim(it.n);
        const uint32_t nMB = Dp > (uint32_t)MT ? Dp / MT : 1u;
        const uint32_t local = t - it.tile0;
        double sc = 1.0 / (double)(1u << it.n);
        if constexpr (PLANES == 2) sc = __builtin_ldexp(sc, -pe[slot]);
        bool staged = false;
        if constexpr (AHEAD > 0) {
            constexpr uint32_t GP = 32 * RB / Pack<PLANES>::SK / 2;   // slice pairs per sign group
            const uint32_t nP = Dp / Pack<PLANES>::SK / 2;
            staged = Dp >= (uint32_t)MT && nP % GP == 0;
            if (staged) {
                // its waits count only its own copies: let the claim return first
                wait_vmcnt<0>();
                contract_tile_lds<PLANES, RB, FORWARD, AHEAD>(ws + it.ws_off, (unsigned char*)it.out, it.n,
                                                              local / nMB, local % nMB, sc, 0, lds);
            }
        }
        if (!staged)
            contract_tile<PLANES, RB, WAVES, FORWARD, PF>(ws + it.ws_off, (unsigned char*)it.out, it.n,
                                                          local / nMB, local % nMB, sc, 0, lds);
        if (threadIdx.x == 0) next = claimed;   // the epilogue ended with a barrier
        __syncthreads();
        t = next;
        __syncthreads();
    }
}

template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0>
__global__ __launch_bounds__(WAVES * 64) void contract_batched_kernel(const BatchItem* __restrict__ items,
                                                                      const uint32_t* __restrict__ tile_slot,
                                                                      uint32_t total,
                                                                      const unsigned char* __restrict__ ws,
                                                                      unsigned int* __restrict__ counter,
                                                                      const int* __restrict__ pe) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ uint32_t next;
    batched_loop<PLANES, RB, WAVES, PF, AHEAD>(items, tile_slot, total, ws, counter, pe, lds, next);
}

// The same loop with the registers budgeted for two waves per SIMD, so that
// a second workgroup's contraction covers one's change-over between tiles.
template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0>
__global__ __launch_bounds__(WAVES * 64, 2) void contract_batched2_kernel(const BatchItem* __restrict__ items,
                                                                          const uint32_t* __restrict__ tile_slot,
                                                                          uint32_t total,
                                                                          const unsigned char* __restrict__ ws,
                                                                          unsigned int* __restrict__ counter,
                                                                          const int* __restrict__ pe) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ uint32_t next;
    batched_loop<PLANES, RB, WAVES, PF, AHEAD>(items, tile_slot, total, ws, counter, pe, lds, next);
}

// Tile shapes the persistent kernel can run with: (RB, WAVES, PF, waves per
// SIMD the registers are budgeted for, LDS-staged pairs ahead or 0).
struct BTile {
    int rb, waves, pf, occ, ahead = 0;
};
// (4 x 32 rows per wave does not fit the persistent loop's registers: its
// accumulators, ring and tile bookkeeping would spill.)
constexpr BTile BTILES[] = {
    {2, 4, 4, 1},     // 1: 256 rows per output tile
    {1, 4, 2, 1},     // 2: 128 rows
    {1, 2, 2, 1},     // 3: 64 rows
    {2, 4, 2, 2},     // 4: 256 rows, shallower ring, two workgroups per CU
    {2, 4, 2, 1, 3},  // 5: 256 rows, LDS-staged 3 pairs ahead (ring for small matrices)
};
constexpr int NBTILES = sizeof(BTILES) / sizeof(BTILES[0]);

template <int PLANES, int RB, int WAVES, int PF, int OCC, int AHEAD = 0>
hipError_t launch_contract_batched(const BatchItem* items, const uint32_t* tile_slot, uint32_t total,
                                   const unsigned char* ws, unsigned int* counter, const int* pe, hipStream_t s) {
    if constexpr (!ring_tile_ok(PLANES, RB)) {
        return hipErrorInvalidValue;
    } else {
        auto launch = [&](auto kern) -> hipError_t {
            const int stage = WAVES * 1024 * 8;
            const int ring = AHEAD > 0 ? (AHEAD + 1) * 2 * Pack<PLANES>::NPL * FRAG : 0;
            const int lds = ring > stage ? ring : stage;
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e != hipSuccess) return e;
            int dev = 0, cus = 0, per_cu = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
                return e;
            if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, WAVES * 64, lds)) !=
                hipSuccess)
                return e;
            if (per_cu < 1) per_cu = 1;
            uint32_t grid = (uint32_t)cus * (uint32_t)per_cu;
            if (grid > total) grid = total;   // never more workgroups than tiles
            hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVES * 64), lds, s, items, tile_slot, total, ws, counter, pe);
            return hipGetLastError();
        };
        if constexpr (OCC == 2) return launch(contract_batched2_kernel<PLANES, RB, WAVES, PF, AHEAD>);
        else return launch(contract_batched_kernel<PLANES, RB, WAVES, PF, AHEAD>);
    }
}

template <int PLANES>
hipError_t launch_contract_btile(int btile, const BatchItem* items, const uint32_t* tile_slot, uint32_t total,
                                 const unsigned char* ws, unsigned int* counter, const int* pe, hipStream_t s) {
    switch (btile) {
        case 1: return launch_contract_batched<PLANES, 2, 4, 4, 1>(items, tile_slot, total, ws, counter, pe, s);
        case 2: return launch_contract_batched<PLANES, 1, 4, 2, 1>(items, tile_slot, total, ws, counter, pe, s);
        case 3: return launch_contract_batched<PLANES, 1, 2, 2, 1>(items, tile_slot, total, ws, counter, pe, s);
        case 4: return launch_contract_batched<PLANES, 2, 4, 2, 2>(items, tile_slot, total, ws, counter, pe, s);
        case 5: return launch_contract_batched<PLANES, 2, 4, 2, 1, 3>(items, tile_slot, total, ws, counter, pe, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int batched_tile_count() { return NBTILES; }

bool batched_tile_valid(int planes, int btile) {
    return btile >= 1 && btile <= NBTILES && ring_tile_ok(planes, BTILES[btile - 1].rb);
}

uint32_t batched_output_tiles(int btile, int n) {
    const BTile t = BTILES[btile - 1];
    const uint32_t MT = t.rb * t.waves * 32;
    const uint32_t Dp = mfma::padded_dim(n);
    return (Dp > MT ? Dp / MT : 1u) * (Dp / mfma::XT);
}

uint32_t batched_pack_tiles(int n) { return mfma::pack_tiles(n); }

size_t batched_packed_bytes(int planes, int n) {
    const size_t Dp = mfma::padded_dim(n);
    const size_t eb = planes == 3 ? mfma::Pack<3>::EB : (planes == 2 ? mfma::Pack<2>::EB : mfma::Pack<1>::EB);
    return Dp * Dp * eb;
}

hipError_t launch_batched(int planes, int btile, const BatchItem* items_dev, const uint32_t* pack_slot_dev,
                          const uint32_t* tile_slot_dev, uint32_t count, uint32_t pack_total, uint32_t tile_total,
                          unsigned char* packed, unsigned int* counter_dev, int* pe_dev, float* partial_dev,
                          hipStream_t stream) {
    if (!batched_tile_valid(planes, btile) || pack_total == 0 || count == 0) return hipErrorInvalidValue;
    if (planes == 2 && (!pe_dev || !partial_dev)) return hipErrorInvalidValue;
    if (planes == 3) {
        hipLaunchKernelGGL((pack_batched_kernel<3>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)nullptr);
    } else if (planes == 2) {
        hipLaunchKernelGGL(absmax_batched_kernel, dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           partial_dev);
        hipLaunchKernelGGL(prescale_batched_kernel, dim3(count), dim3(256), 0, stream, items_dev,
                           (const float*)partial_dev, pe_dev);
        hipLaunchKernelGGL((pack_batched_kernel<2>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)pe_dev);
    } else {
        hipLaunchKernelGGL((pack_batched_kernel<1>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)nullptr);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int* pe = pe_dev;
    if (planes == 3)
        return launch_contract_btile<3>(btile, items_dev, tile_slot_dev, tile_total, packed, counter_dev, pe, stream);
    if (planes == 2)
        return launch_contract_btile<2>(btile, items_dev, tile_slot_dev, tile_total, packed, counter_dev, pe, stream);
    return launch_contract_btile<1>(btile, items_dev, tile_slot_dev, tile_total, packed, counter_dev, pe, stream);
}

}  // namespace pauli
