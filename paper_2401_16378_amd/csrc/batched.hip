// Uneven batch: many matrices of different order decomposed by one batched
// pack launch and one persistent contraction launch (the paper's embarrassing
// parallelism over coefficients, section 3, extended over matrices).
//
// The host builds a descriptor table in device memory: one entry per matrix,
// in decreasing order of N (longest-processing-time first), with the matrix's
// packed-operand offset and its first pack tile and first output tile in the
// batch-wide numbering, followed by the slot of every pack tile and of every
// output tile, and the output tiles' queues.  A pack workgroup finds its
// matrix with one read of the pack slot table.  The contraction kernel is
// persistent: each workgroup takes output tiles from its queue's atomic
// counter until the queue is exhausted, so every workgroup ends once its
// counter passes the queue's last tile and the grid drains.  There are up to
// eight queues, a workgroup's queue being its index modulo the queue count:
// workgroups are dispatched to the eight XCDs round-robin, so each queue is
// served by one XCD, and the host puts all row blocks of a flip-mask slab in
// one queue (slabs dealt to the least loaded queue by estimated cost, largest
// first), so that a slab's packed operand is fetched into one XCD's L2 and
// reused there.  (Under another dispatch order every tile is still taken
// exactly once; only the reuse depends on it.)  A workgroup claims its next
// tile when it starts the current one (the atomic's round trip then overlaps
// the contraction) and finds a tile's matrix with one read of the output slot
// table.  The pack kernel's first threads zero the counters: the contraction
// runs after the pack on the same stream, and the previous contraction has
// finished before the pack starts (no memset node, so the sequence can be
// captured in a HIP graph and replayed).  The two-plane split first finds
// every matrix's prescale: one reduction workgroup per pack tile takes the
// largest component of an equal share of its matrix, then one workgroup per
// matrix reduces its shares.
#include "mfma_tile.hpp"

namespace pauli {
namespace {

using namespace mfma;

// Queue counters for a fused contraction (no pack kernel to clear them).
__global__ __launch_bounds__(64) void clear_counters_kernel(unsigned int* __restrict__ counter) {
    if (threadIdx.x < MAX_QUEUES) counter[threadIdx.x] = 0u;
}

// Share t of its matrix (pack tile t): 4^n / pack_tiles(n) consecutive
// elements, an even count (32 x 128 for n >= 7, the whole matrix below 5;
// the batch has n >= 1).
__global__ __launch_bounds__(256) void absmax_batched_kernel(const BatchItem* __restrict__ items,
                                                             const uint32_t* __restrict__ pack_slot,
                                                             float* __restrict__ partial) {
    __shared__ float red[4];
    const BatchItem it = items[pack_slot[blockIdx.x]];
    const uint32_t n = 1u << (2 * it.n);
    const uint32_t per = n / pack_tiles(it.n);    // even (n >= 4), so whole 16-byte pairs
    const float4* p = (const float4*)((const float2*)it.in + (size_t)(blockIdx.x - it.pack0) * per);
    float m = 0.f;
#pragma unroll 4
    for (uint32_t i = threadIdx.x; i < per / 2; i += 256) {
        const float4 v = p[i];
        m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(v.x), __builtin_fabsf(v.y)),
                                               __builtin_fmaxf(__builtin_fabsf(v.z), __builtin_fabsf(v.w))));
    }
    m = block_max256(m, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// One workgroup per descriptor slot: the matrix's prescale exponent.  With
// `counter` set (a fused contraction follows, with no pack kernel) the first
// workgroup also clears the queue counters.
__global__ __launch_bounds__(256) void prescale_batched_kernel(const BatchItem* __restrict__ items,
                                                               const float* __restrict__ partial,
                                                               int* __restrict__ pe,
                                                               unsigned int* __restrict__ counter) {
    __shared__ float red[4];
    if (counter && blockIdx.x == 0 && threadIdx.x < MAX_QUEUES) counter[threadIdx.x] = 0u;
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
    if (blockIdx.x == 0 && threadIdx.x < MAX_QUEUES) counter[threadIdx.x] = 0u;   // for the contraction that follows
    const uint32_t slot = pack_slot[blockIdx.x];
    const BatchItem it = items[slot];
    pack_tile<PLANES, FORWARD, false>((const unsigned char*)it.in, ws + it.ws_off, it.n,
                                      blockIdx.x - it.pack0, lds, PLANES == 2 ? pe[slot] : 0);
}

// Bytes of one LDS staging tile of a fused contraction chunk of KC <= 128 K
// values (the pack's layout).
template <int PLANES, int KC>
constexpr int fused_stage_bytes() {
    static_assert(KC == 64 || KC == 128, "a chunk is one or two 32 x 64 halves of a pack tile");
    return Pack<PLANES>::NPL * XT * (KC * Pack<PLANES>::ESZ + 16);
}

// Fused output tile of the batch: 32 flip masks x MT rows (MT = 4 RB 32) of
// the matrix at src, gathering and splitting its operand itself instead of
// reading a packed operand.  The K range is walked in chunks of KT <= 128
// values; for each chunk every thread of the four waves loads one 4x4
// micro-block of G (load_block_fwd) and stages its split in one of two LDS
// tiles (stage_block, the pack's layout), from which each wave reads its B
// fragments.  The next chunk's micro-blocks are requested before the current
// chunk's MFMAs and staged after them; one barrier per chunk.  The split, the
// staged values and the order of every accumulation are the separate pack's
// and contraction's, so the result is theirs bit for bit.
template <int PLANES, int RB, int KC>
__device__ __attribute__((always_inline)) inline void fused_tile(const unsigned char* __restrict__ src,
                                                                 unsigned char* __restrict__ dst, int N, uint32_t xb,
                                                                 uint32_t mb, double scale, int pe,
                                                                 unsigned char* lds) {
    using P = Pack<PLANES>;
    constexpr int ACC = P::ACC;
    constexpr int MT = 4 * RB * 32;
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)KC ? Dp : (uint32_t)KC;
    const uint32_t pitch = KT * P::ESZ + 16, PS = XT * pitch;
    const uint32_t nKT = Dp / KT, SPC = KT / P::SK;      // chunks, slices per chunk
    const uint32_t X0 = xb * XT;
    const bool full = D >= 32u;
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));   // per call, as in store_tile
    const bool loader = (uint32_t)tid < 2 * KT;           // threads that own a micro-block of a chunk
    const int g = tid >> 6, w6 = tid & 63;
    const int lane = tid & 63, wave = tid >> 6, l32 = lane & 31, h = lane >> 5;
    const uint32_t Pw = mb * MT + wave * RB * 32;
    const bool active = Pw < Dp;                          // waves past the padded order only stage

    uint32_t fA[2][4];
    float fF[4][4];
    if constexpr (PLANES >= 2) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t q0 = 16 * e + 8 * h + 2 * jj;
                const uint32_t s0 = ONE16<PLANES> | ((__popc(l32 & q0) & 1) ? 0x8000u : 0u);
                const uint32_t s1 = ONE16<PLANES> | ((__popc(l32 & (q0 + 1)) & 1) ? 0x8000u : 0u);
                fA[e][jj] = s0 | (s1 << 16);
            }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                fF[e][t] = (__popc(l32 & (8 * e + 4 * h + t)) & 1) ? -1.f : 1.f;
    }
    f32x16 acc[ACC][RB][2], tot[1][RB][2];
#pragma unroll
    for (int a = 0; a < ACC; ++a)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][rb][cb][r] = tot[0][rb][cb][r] = 0.f;

    f32x2 v[16];
    int xh = 0, kh = 0;
    if (loader) {
        load_block_fwd<false>(src, D, full, X0, 0u, g, w6, v, xh, kh);
        stage_block<PLANES, FORWARD>(v, xh, kh, pe, lds, pitch);
    }
    __syncthreads();
    for (uint32_t kt = 0; kt < nKT; ++kt) {
        const unsigned char* cur = lds + (kt & 1u) * (uint32_t)fused_stage_bytes<PLANES, KC>();
        unsigned char* nxt = lds + ((kt + 1u) & 1u) * (uint32_t)fused_stage_bytes<PLANES, KC>();
        const bool more = kt + 1 < nKT;
        if (more && loader) load_block_fwd<false>(src, D, full, X0, (kt + 1) * KT, g, w6, v, xh, kh);
        if (active) {
            for (uint32_t s = 0; s < SPC; ++s) {
                const uint32_t S = kt * SPC + s;                 // slice index along K
                u32x4 B[P::NPL];
                const unsigned char* fb = cur + l32 * pitch + (s * P::SK + h * (P::SK / 2)) * P::ESZ;
#pragma unroll
                for (int f = 0; f < P::NPL; ++f) B[f] = *(const u32x4*)(fb + f * PS);
                const uint32_t qblk = (S * P::SK) >> 5;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const bool neg = __popc(((Pw >> 5) + rb) & qblk) & 1;
                    if constexpr (PLANES >= 2) {
                        const uint32_t m = neg ? 0x80008000u : 0u;
                        const int e = S & 1;
                        const u32x4 A = u32x4{fA[e][0] ^ m, fA[e][1] ^ m, fA[e][2] ^ m, fA[e][3] ^ m};
#pragma unroll
                        for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                            for (int cb = 0; cb < 2; ++cb)
                                acc[pl == 0 ? 0 : ACC - 1][rb][cb] =
                                    mfma16<PLANES>(A, B[pl * 2 + cb], acc[pl == 0 ? 0 : ACC - 1][rb][cb]);
                    } else {
                        const f32x4 B0 = __builtin_bit_cast(f32x4, B[0]), B1 = __builtin_bit_cast(f32x4, B[1]);
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const float A = (neg ? -1.f : 1.f) * fF[S & 3][t];
                            acc[0][rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B0[t], acc[0][rb][0], 0, 0, 0);
                            acc[0][rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B1[t], acc[0][rb][1], 0, 0, 0);
                        }
                    }
                }
                if constexpr (PLANES == 1) {
                    if ((S + 1) % FLUSH_SLICES == 0) flush_into<RB>(tot, acc);
                }
            }
        }
        if (more && loader) stage_block<PLANES, FORWARD>(v, xh, kh, pe, nxt, pitch);
        __syncthreads();   // chunk kt + 1 staged; chunk kt read by every wave
    }
    if constexpr (PLANES == 1) {
        flush_into<RB>(tot, acc);
        store_tile<PLANES, RB, FORWARD>(tot, dst, N, X0, Pw, scale, 0, lds);
    } else {
        store_tile<PLANES, RB, FORWARD>(acc, dst, N, X0, Pw, scale, 0, lds);
    }
}

// AHEAD > 0: output tiles of matrices with at least MT rows and a whole
// number of sign groups of slice pairs take the LDS-staged contraction
// (each fragment copied once per workgroup, AHEAD pairs ahead); smaller ones
// take the register ring.  FUSED > 0: every tile gathers and splits its own
// operand (fused_tile) in chunks of FUSED K values; there is no packed
// operand.
// queues = [nq | nq + 1 offsets | tile ids]: queue q holds the output tiles
// queues[2 + nq + j] for queues[1 + q] <= j < queues[2 + q]; counter[q] is
// its claim counter.
template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0, int FUSED = 0>
__device__ __attribute__((always_inline)) inline void batched_loop(const BatchItem* __restrict__ items,
                                                                   const uint32_t* __restrict__ tile_slot,
                                                                   const uint32_t* __restrict__ queues,
                                                                   const unsigned char* __restrict__ ws,
                                                                   unsigned int* __restrict__ counter,
                                                                   const int* __restrict__ pe,
                                                                   unsigned char* lds, uint32_t& next) {
    static_assert(AHEAD == 0 || WAVES == 4, "the LDS-staged contraction runs four waves per workgroup");
    static_assert(!FUSED || (WAVES == 4 && AHEAD == 0), "the fused contraction runs four waves per workgroup");
    constexpr int MT = WAVES * RB * 32;
    const uint32_t nq = queues[0];
    const uint32_t q = blockIdx.x % nq;
    const uint32_t qbeg = queues[1 + q], qlen = queues[2 + q] - qbeg;
    const uint32_t* qtiles = queues + 2 + nq + qbeg;
    unsigned int* qcount = counter + q;
    if (threadIdx.x == 0) next = atomicAdd(qcount, 1u);
    __syncthreads();
    uint32_t j = next;
    __syncthreads();                   // everyone has read `next` before it is rewritten
    while (j < qlen) {                 // uniform: every workgroup leaves once its queue is done
        uint32_t claimed = 0;
        if (threadIdx.x == 0) claimed = atomicAdd(qcount, 1u);   // read only after this tile
        const uint32_t t = qtiles[j];
        const uint32_t slot = tile_slot[t];
        const BatchItem it = items[slot];
        const uint32_t Dp = padded_dim(it.n);
        const uint32_t nMB = Dp > (uint32_t)MT ? Dp / MT : 1u;
        const uint32_t local = t - it.tile0;
        double sc = 1.0 / (double)(1u << it.n);
        if constexpr (PLANES == 2) sc = __builtin_ldexp(sc, -pe[slot]);
        if constexpr (FUSED) {
            fused_tile<PLANES, RB, FUSED>((const unsigned char*)it.in, (unsigned char*)it.out, it.n, local / nMB,
                                          local % nMB, sc, PLANES == 2 ? pe[slot] : 0, lds);
        } else {
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
        }
        if (threadIdx.x == 0) next = claimed;   // the epilogue ended with a barrier
        __syncthreads();
        j = next;
        __syncthreads();
    }
}

template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0, int FUSED = 0>
__global__ __launch_bounds__(WAVES * 64) void contract_batched_kernel(const BatchItem* __restrict__ items,
                                                                      const uint32_t* __restrict__ tile_slot,
                                                                      const uint32_t* __restrict__ queues,
                                                                      const unsigned char* __restrict__ ws,
                                                                      unsigned int* __restrict__ counter,
                                                                      const int* __restrict__ pe) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ uint32_t next;
    batched_loop<PLANES, RB, WAVES, PF, AHEAD, FUSED>(items, tile_slot, queues, ws, counter, pe, lds, next);
}

// The same loop with the registers budgeted for two waves per SIMD, so that
// a second workgroup's contraction covers one's change-over between tiles.
template <int PLANES, int RB, int WAVES, int PF, int AHEAD = 0, int FUSED = 0>
__global__ __launch_bounds__(WAVES * 64, 2) void contract_batched2_kernel(const BatchItem* __restrict__ items,
                                                                          const uint32_t* __restrict__ tile_slot,
                                                                      const uint32_t* __restrict__ queues,
                                                                          const unsigned char* __restrict__ ws,
                                                                          unsigned int* __restrict__ counter,
                                                                          const int* __restrict__ pe) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ uint32_t next;
    batched_loop<PLANES, RB, WAVES, PF, AHEAD, FUSED>(items, tile_slot, queues, ws, counter, pe, lds, next);
}

// Tile shapes the persistent kernel can run with: (RB, WAVES, PF, waves per
// SIMD the registers are budgeted for, LDS-staged pairs ahead or 0, fused
// chunk or 0).  Fused shapes gather and split their operand themselves
// (fused_tile) in chunks of that many K values: the launch sequence has no
// pack kernel.
struct BTile {
    int rb, waves, pf, occ, ahead = 0, fused = 0;
};
// (4 x 32 rows per wave does not fit the persistent loop's registers: its
// accumulators, ring and tile bookkeeping would spill.)
constexpr BTile BTILES[] = {
    {2, 4, 4, 1},     // 1: 256 rows per output tile
    {1, 4, 2, 1},     // 2: 128 rows
    {1, 2, 2, 1},     // 3: 64 rows
    {2, 4, 2, 2},     // 4: 256 rows, shallower ring, two workgroups per CU
    {2, 4, 2, 1, 3},  // 5: 256 rows, LDS-staged 3 pairs ahead (ring for small matrices)
    {2, 4, 0, 1, 0, 128},    // 6: 256 rows, fused gather/split/contract, 128-value chunks
    {4, 4, 0, 1, 0, 128},    // 7: 512 rows, fused
    {2, 4, 0, 2, 0, 128},    // 8: 256 rows, fused, registers for two workgroups per CU
    {2, 4, 0, 2, 0, 64},     // 9: 256 rows, fused, 64-value chunks (LDS for two workgroups per CU)
};
constexpr int NBTILES = sizeof(BTILES) / sizeof(BTILES[0]);

// A fused 4 x 32-row-per-wave tile fits the register file only with the
// two-plane split's smaller operand (the binary32 plane adds its flushed
// total, the three-plane split six fragments per slice: both would spill).
constexpr bool fused_ok(int planes, int rb) { return rb != 4 || planes == 2; }

template <int PLANES, int RB, int WAVES, int PF, int OCC, int AHEAD = 0, int FUSED = 0>
hipError_t launch_contract_batched(const BatchItem* items, const uint32_t* tile_slot, const uint32_t* queues,
                                   uint32_t total, const unsigned char* ws, unsigned int* counter, const int* pe,
                                   hipStream_t s) {
    if constexpr (FUSED > 0 ? !fused_ok(PLANES, RB) : !ring_tile_ok(PLANES, RB)) {
        return hipErrorInvalidValue;
    } else {
        auto launch = [&](auto kern) -> hipError_t {
            const int stage = WAVES * 1024 * 8;
            int ring = AHEAD > 0 ? (AHEAD + 1) * 2 * Pack<PLANES>::NPL * FRAG : 0;
            if constexpr (FUSED > 0) ring = 2 * fused_stage_bytes<PLANES, FUSED>();
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
            if (grid > total) grid = total;   // never more workgroups than tiles (nor fewer than queues)
            hipLaunchKernelGGL(kern, dim3(grid), dim3(WAVES * 64), lds, s, items, tile_slot, queues, ws, counter, pe);
            return hipGetLastError();
        };
        if constexpr (OCC == 2) return launch(contract_batched2_kernel<PLANES, RB, WAVES, PF, AHEAD, FUSED>);
        else return launch(contract_batched_kernel<PLANES, RB, WAVES, PF, AHEAD, FUSED>);
    }
}

template <int PLANES>
hipError_t launch_contract_btile(int btile, const BatchItem* items, const uint32_t* tile_slot, const uint32_t* queues,
                                 uint32_t total, const unsigned char* ws, unsigned int* counter, const int* pe,
                                 hipStream_t s) {
    const uint32_t* q = queues;
    switch (btile) {
        case 1: return launch_contract_batched<PLANES, 2, 4, 4, 1>(items, tile_slot, q, total, ws, counter, pe, s);
        case 2: return launch_contract_batched<PLANES, 1, 4, 2, 1>(items, tile_slot, q, total, ws, counter, pe, s);
        case 3: return launch_contract_batched<PLANES, 1, 2, 2, 1>(items, tile_slot, q, total, ws, counter, pe, s);
        case 4: return launch_contract_batched<PLANES, 2, 4, 2, 2>(items, tile_slot, q, total, ws, counter, pe, s);
        case 5: return launch_contract_batched<PLANES, 2, 4, 2, 1, 3>(items, tile_slot, q, total, ws, counter, pe, s);
        case 6:
            return launch_contract_batched<PLANES, 2, 4, 0, 1, 0, 128>(items, tile_slot, q, total, ws, counter, pe, s);
        case 7:
            return launch_contract_batched<PLANES, 4, 4, 0, 1, 0, 128>(items, tile_slot, q, total, ws, counter, pe, s);
        case 8:
            return launch_contract_batched<PLANES, 2, 4, 0, 2, 0, 128>(items, tile_slot, q, total, ws, counter, pe, s);
        case 9:
            return launch_contract_batched<PLANES, 2, 4, 0, 2, 0, 64>(items, tile_slot, q, total, ws, counter, pe, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int batched_tile_count() { return NBTILES; }

// Untuned shape: fused, registers for two workgroups per CU; the three-plane
// split needs the 64-value chunks for its staging to fit twice in LDS.
int batched_default_tile(int planes) { return planes == 3 ? 9 : 8; }

bool batched_tile_valid(int planes, int btile) {
    if (btile < 1 || btile > NBTILES) return false;
    const BTile t = BTILES[btile - 1];
    return t.fused > 0 ? fused_ok(planes, t.rb) : ring_tile_ok(planes, t.rb);
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
                          const uint32_t* tile_slot_dev, const uint32_t* queues_dev, uint32_t count,
                          uint32_t pack_total, uint32_t tile_total, unsigned char* packed, unsigned int* counter_dev,
                          int* pe_dev, float* partial_dev, hipStream_t stream) {
    if (!batched_tile_valid(planes, btile) || pack_total == 0 || count == 0) return hipErrorInvalidValue;
    if (planes == 2 && (!pe_dev || !partial_dev)) return hipErrorInvalidValue;
    const bool fused = BTILES[btile - 1].fused > 0;
    if (planes == 2) {
        hipLaunchKernelGGL(absmax_batched_kernel, dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           partial_dev);
        hipLaunchKernelGGL(prescale_batched_kernel, dim3(count), dim3(256), 0, stream, items_dev,
                           (const float*)partial_dev, pe_dev, fused ? counter_dev : nullptr);
    }
    if (fused && planes != 2) {
        hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, stream, counter_dev);
    } else if (fused) {
        // the prescale kernel cleared the counters
    } else if (planes == 3) {
        hipLaunchKernelGGL((pack_batched_kernel<3>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)nullptr);
    } else if (planes == 2) {
        hipLaunchKernelGGL((pack_batched_kernel<2>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)pe_dev);
    } else {
        hipLaunchKernelGGL((pack_batched_kernel<1>), dim3(pack_total), dim3(256), 0, stream, items_dev, pack_slot_dev,
                           packed, counter_dev, (const int*)nullptr);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int* pe = pe_dev;
    const uint32_t* qd = queues_dev;
    if (planes == 3)
        return launch_contract_btile<3>(btile, items_dev, tile_slot_dev, qd, tile_total, packed, counter_dev, pe, stream);
    if (planes == 2)
        return launch_contract_btile<2>(btile, items_dev, tile_slot_dev, qd, tile_total, packed, counter_dev, pe, stream);
    return launch_contract_btile<1>(btile, items_dev, tile_slot_dev, qd, tile_total, packed, counter_dev, pe, stream);
}

}  // namespace pauli
