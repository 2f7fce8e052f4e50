// Single-matrix entry of the matrix-core path (see mfma_tile.hpp for the
// method): one pack launch over all pack tiles of the batch of equal-order
// matrices, then one contraction launch over all output tiles.
#include "mfma_tile.hpp"

namespace pauli {
namespace {

using namespace mfma;

// pe: prescale exponent of each matrix of the batch (two-plane split only).
template <int PLANES, int DIR, bool IN128>
__global__ __launch_bounds__(256) void pack_kernel(const void* __restrict__ in, void* __restrict__ ws, int N,
                                                   const int* __restrict__ pe) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[pack_lds_bytes<PLANES, DIR>()];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    pack_tile<PLANES, DIR, IN128>(src, wsm, N, blockIdx.x, lds, PLANES == 2 ? pe[blockIdx.y] : 0);
}

// Pack for the Hermitian contraction: the K ranges its half walk skips are not packed.
template <int PLANES, bool IN128>
__global__ __launch_bounds__(256) void pack_herm_kernel(const void* __restrict__ in, void* __restrict__ ws, int N,
                                                        uint32_t hmin, const int* __restrict__ pe) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[pack_lds_bytes<PLANES>()];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    pack_tile<PLANES, FORWARD, IN128>(src, wsm, N, herm_pack_tile(N, hmin, blockIdx.x), lds,
                                      PLANES == 2 ? pe[blockIdx.y] : 0);
}

// ---- prescale of the two-plane split ----
// Largest |re|, |im| of each matrix (as binary32, the precision the pack
// reads), in two launches: absmax_kernel reduces R contiguous ranges of the
// 4^N elements of matrix blockIdx.y to R partial maxima, prescale_kernel
// reduces those and stores the matrix's prescale exponent.  Both write every
// value they produce, so the workspace needs no clearing.
template <bool IN128>
__global__ __launch_bounds__(256) void absmax_kernel(const void* __restrict__ in, int N, float* __restrict__ partial,
                                                     uint32_t R) {
    __shared__ float red[4];
    const size_t n = (size_t)1 << (2 * N);            // elements per matrix
    const size_t per = n / R;                          // R divides n; per is even unless N = 0
    const size_t lo = (size_t)blockIdx.x * per;
    float m = 0.f;
    if constexpr (IN128) {
        const double2* p = (const double2*)in + (size_t)blockIdx.y * n + lo;
        for (size_t i = threadIdx.x; i < per; i += 256) {
            const double2 v = p[i];
            m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf((float)v.x), __builtin_fabsf((float)v.y)));
        }
    } else if (per % 2 == 0) {
        const float4* p = (const float4*)((const float2*)in + (size_t)blockIdx.y * n + lo);
        for (size_t i = threadIdx.x; i < per / 2; i += 256) {
            const float4 v = p[i];
            m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(v.x), __builtin_fabsf(v.y)),
                                                   __builtin_fmaxf(__builtin_fabsf(v.z), __builtin_fabsf(v.w))));
        }
    } else {
        const float2* p = (const float2*)in + (size_t)blockIdx.y * n + lo;
        for (size_t i = threadIdx.x; i < per; i += 256) {
            const float2 v = p[i];
            m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf(v.x), __builtin_fabsf(v.y)));
        }
    }
    m = block_max256(m, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * R + blockIdx.x] = m;
}

// Hermitian input: |G[c][r]| = |G[r][c]|, so the largest component lies in
// the lower triangle (diagonal included).  Block b reads, for each of its
// row pairs (r, D-1-r), the D + 1 elements G[r][0..r] and G[D-1-r][0..D-1-r]:
// half of G, the same maximum.  Needs D >= 2; R divides D / 2.
template <bool IN128>
__global__ __launch_bounds__(256) void absmax_lower_kernel(const void* __restrict__ in, int N,
                                                           float* __restrict__ partial, uint32_t R) {
    __shared__ float red[4];
    const uint32_t D = 1u << N;
    const uint32_t ppb = (D / 2u) / R;                 // row pairs per block
    const size_t mat = (size_t)D * D;
    float m = 0.f;
    for (uint32_t pp = 0; pp < ppb; ++pp) {
        const uint32_t r = blockIdx.x * ppb + pp;      // rows r and D-1-r: r + 1 and D - r elements
        for (uint32_t e = threadIdx.x; e <= D; e += 256) {
            const size_t idx = e <= r ? (size_t)r * D + e : (size_t)(D - 1u - r) * D + (e - r - 1u);
            float a, b;
            if constexpr (IN128) {
                const double2 v = ((const double2*)in)[(size_t)blockIdx.y * mat + idx];
                a = (float)v.x;
                b = (float)v.y;
            } else {
                const float2 v = ((const float2*)in)[(size_t)blockIdx.y * mat + idx];
                a = v.x;
                b = v.y;
            }
            m = __builtin_fmaxf(m, __builtin_fmaxf(__builtin_fabsf(a), __builtin_fabsf(b)));
        }
    }
    m = block_max256(m, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * R + blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void prescale_kernel(const float* __restrict__ partial, uint32_t R,
                                                       int* __restrict__ pe) {
    __shared__ float red[4];
    float m = 0.f;
    for (uint32_t i = threadIdx.x; i < R; i += 256) m = __builtin_fmaxf(m, partial[(size_t)blockIdx.x * R + i]);
    m = block_max256(m, red);
    if (threadIdx.x == 0) pe[blockIdx.x] = prescale_exponent(m);
}

struct Params {
    const void* ws;
    void* out;
    int N;
    int out128;
    double scale;
    const int* pe;   // prescale exponents (two-plane split), else unused
};

// The output scale of matrix blockIdx.y: the two-plane split undoes its prescale here.
template <int PLANES>
__device__ inline double out_scale(const Params& prm) {
    if constexpr (PLANES == 2) return __builtin_ldexp(prm.scale, -prm.pe[blockIdx.y]);
    else return prm.scale;
}

template <int PLANES, int RB, int WAVES, int DIR, int PF, bool HERM = false>
__global__ __launch_bounds__(WAVES * 64 > 256 ? WAVES * 64 : 256) void contract_kernel(Params prm) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    constexpr int MT = WAVES * RB * 32;
    const uint32_t D = 1u << prm.N, Dp = padded_dim(prm.N);
    const uint32_t nMB = Dp / MT;
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const unsigned char* wsm = (const unsigned char*)prm.ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    unsigned char* dst = (unsigned char*)prm.out + (size_t)blockIdx.y * D * D * (prm.out128 ? 16 : 8);
    uint32_t xb = L / nMB;
    if constexpr (HERM) {
        // The Hermitian walk halves K only for xb >= (step K) / 32, so the
        // first slabs cost twice as much: deal slabs to the XCDs round-robin
        // (XCD k, which owns the slab range [k S, k S + S), gets slabs
        // k, k + 8, ...) instead of in ranges, one long slab per XCD, first.
        const uint32_t nXB = Dp / XT;
        if ((gridDim.x & 7u) == 0 && (nXB & 7u) == 0) {
            const uint32_t S = nXB >> 3;
            xb = (xb % S) * 8 + xb / S;
        }
    }
    contract_tile<PLANES, RB, WAVES, DIR, PF, HERM>(wsm, dst, prm.N, xb, L % nMB, out_scale<PLANES>(prm), prm.out128,
                                                    lds);
}

template <int PLANES, int RB, int DIR, int AHEAD>
__global__ __launch_bounds__(256) void contract_lds_kernel(Params prm) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    constexpr int MT = 4 * RB * 32;
    const uint32_t D = 1u << prm.N, Dp = padded_dim(prm.N);
    const uint32_t nMB = Dp / MT;
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const unsigned char* wsm = (const unsigned char*)prm.ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    unsigned char* dst = (unsigned char*)prm.out + (size_t)blockIdx.y * D * D * (prm.out128 ? 16 : 8);
    contract_tile_lds<PLANES, RB, DIR, AHEAD>(wsm, dst, prm.N, L / nMB, L % nMB, out_scale<PLANES>(prm),
                                              prm.out128, lds);
}

template <int PLANES, int RB, int AHEAD, int DIR>
hipError_t launch_contract_lds(const Params& p, int batch, hipStream_t s) {
    constexpr int MT = 4 * RB * 32;
    const uint32_t Dp = padded_dim(p.N);
    const uint32_t nMB = Dp / MT, nXB = Dp / XT;
    auto kern = contract_lds_kernel<PLANES, RB, DIR, AHEAD>;
    const int ring = (AHEAD + 1) * 2 * Pack<PLANES>::NPL * FRAG;
    const int stage = 4 * 1024 * (p.out128 ? 16 : 8);
    const int lds = ring > stage ? ring : stage;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nMB * nXB, batch), dim3(256), lds, s, p);
    return hipGetLastError();
}

// ---- tile table: (rows per wave / 32, waves per workgroup, ring depth) ----
struct TileDesc {
    int rb, waves, pf;
    bool lds = false;   // LDS-staged variant (pf = pairs copied ahead)
};
constexpr TileDesc TILES[] = {
    {4, 4, 4},  // 1: 512 rows
    {4, 2, 4},  // 2: 256 rows
    {2, 4, 4},  // 3: 256 rows
    {2, 8, 2},  // 4: 512 rows, two waves per SIMD
    {1, 1, 2},  // 5: 32 rows (zero-padded below 32)
    {1, 4, 2},  // 6: 128 rows
    {4, 1, 4},  // 7: 128 rows
    {2, 2, 4},  // 8: 128 rows
    {1, 2, 2},  // 9: 64 rows
    {4, 4, 8},  // 10: 512 rows, deeper ring
    {4, 2, 8},  // 11: 256 rows, deeper ring
    {2, 4, 8},  // 12: 256 rows, deeper ring
    {4, 4, 3, true},  // 13: 512 rows, LDS-staged, copies 3 slice pairs ahead
    {4, 4, 7, true},  // 14: 512 rows, LDS-staged, copies 7 slice pairs ahead
    {2, 4, 3, true},  // 15: 256 rows, LDS-staged, copies 3 slice pairs ahead
};
constexpr int NTILES = sizeof(TILES) / sizeof(TILES[0]);

template <int PLANES, int RB, int WAVES, int PF, int DIR, bool HERM = false>
hipError_t launch_contract(const Params& p, int batch, hipStream_t s) {
    if constexpr (!ring_tile_ok(PLANES, RB)) {
        return hipErrorInvalidValue;
    } else {
        constexpr int MT = WAVES * RB * 32;
        const uint32_t Dp = padded_dim(p.N);
        const uint32_t nMB = Dp / MT, nXB = Dp / XT;
        auto kern = contract_kernel<PLANES, RB, WAVES, DIR, PF, HERM>;
        // Hermitian: a second output stage for the partner rows, where it fits
        const int lds = WAVES * 1024 * (p.out128 ? 16 : 8) * (HERM && herm_pair_stage_fits(WAVES, p.out128) ? 2 : 1);
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nMB * nXB, batch), dim3(WAVES * 64), lds, s, p);
        return hipGetLastError();
    }
}

// HERM: the Hermitian forward contraction, register-ring tiles only.
template <int PLANES, int DIR, bool HERM = false>
hipError_t launch_tile(int tile, const Params& p, int batch, hipStream_t s) {
    switch (tile) {
        case 1: return launch_contract<PLANES, 4, 4, 4, DIR, HERM>(p, batch, s);
        case 2: return launch_contract<PLANES, 4, 2, 4, DIR, HERM>(p, batch, s);
        case 3: return launch_contract<PLANES, 2, 4, 4, DIR, HERM>(p, batch, s);
        case 4: return launch_contract<PLANES, 2, 8, 2, DIR, HERM>(p, batch, s);
        case 5: return launch_contract<PLANES, 1, 1, 2, DIR, HERM>(p, batch, s);
        case 6: return launch_contract<PLANES, 1, 4, 2, DIR, HERM>(p, batch, s);
        case 7: return launch_contract<PLANES, 4, 1, 4, DIR, HERM>(p, batch, s);
        case 8: return launch_contract<PLANES, 2, 2, 4, DIR, HERM>(p, batch, s);
        case 9: return launch_contract<PLANES, 1, 2, 2, DIR, HERM>(p, batch, s);
        case 10: return launch_contract<PLANES, 4, 4, 8, DIR, HERM>(p, batch, s);
        case 11: return launch_contract<PLANES, 4, 2, 8, DIR, HERM>(p, batch, s);
        case 12: return launch_contract<PLANES, 2, 4, 8, DIR, HERM>(p, batch, s);
        default: break;
    }
    if constexpr (!HERM) {
        switch (tile) {
            case 13: return launch_contract_lds<PLANES, 4, 3, DIR>(p, batch, s);
            case 14: return launch_contract_lds<PLANES, 4, 7, DIR>(p, batch, s);
            case 15: return launch_contract_lds<PLANES, 2, 3, DIR>(p, batch, s);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

// Reduction blocks per matrix for the prescale: a power of two dividing
// 4^N, one per 4096 elements, at most 1024.
uint32_t absmax_blocks(int N) {
    const int lg = 2 * N - 12;
    return lg <= 0 ? 1u : (lg >= 10 ? 1024u : 1u << lg);
}

size_t packed_bytes(int planes, int N, int batch) {
    const size_t Dp = padded_dim(N);
    const size_t eb = planes == 3 ? Pack<3>::EB : (planes == 2 ? Pack<2>::EB : Pack<1>::EB);
    return Dp * Dp * eb * (size_t)batch;
}

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Two-plane workspace: [packed operands | prescale exponents (int per
// matrix) | partial maxima (absmax_blocks(N) floats per matrix)].
int* prescale_exponents(void* ws, int N, int batch) {
    return (int*)((unsigned char*)ws + packed_bytes(2, N, batch));
}
float* prescale_partials(void* ws, int N, int batch) {
    return (float*)((unsigned char*)prescale_exponents(ws, N, batch) + round256(sizeof(int) * (size_t)batch));
}

hipError_t launch_prescale(const void* in, bool in128, void* ws, int N, int batch, hipStream_t s) {
    const uint32_t R = absmax_blocks(N);
    float* partial = prescale_partials(ws, N, batch);
    if (in128) hipLaunchKernelGGL((absmax_kernel<true>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    else hipLaunchKernelGGL((absmax_kernel<false>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    hipLaunchKernelGGL(prescale_kernel, dim3(batch), dim3(256), 0, s, (const float*)partial, R,
                       prescale_exponents(ws, N, batch));
    return hipGetLastError();
}

// The same exponents for Hermitian G from the lower triangle only.
hipError_t launch_prescale_hermitian(const void* in, bool in128, void* ws, int N, int batch, hipStream_t s) {
    const uint32_t D = 1u << N;
    if (D < 2u) return launch_prescale(in, in128, ws, N, batch, s);
    uint32_t R = absmax_blocks(N);                     // a power of two, as is D / 2
    if (R > D / 2u) R = D / 2u;
    float* partial = prescale_partials(ws, N, batch);
    if (in128) hipLaunchKernelGGL((absmax_lower_kernel<true>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    else hipLaunchKernelGGL((absmax_lower_kernel<false>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    hipLaunchKernelGGL(prescale_kernel, dim3(batch), dim3(256), 0, s, (const float*)partial, R,
                       prescale_exponents(ws, N, batch));
    return hipGetLastError();
}

template <int PLANES, int DIR>
hipError_t launch_pack(const void* in, bool in128, void* ws, int N, int batch, hipStream_t s) {
    const int* pe = nullptr;
    if constexpr (PLANES == 2) {
        const hipError_t e = launch_prescale(in, in128, ws, N, batch, s);
        if (e != hipSuccess) return e;
        pe = prescale_exponents(ws, N, batch);
    }
    const dim3 grid(pack_tiles(N), batch);
    if (in128) hipLaunchKernelGGL((pack_kernel<PLANES, DIR, true>), grid, dim3(256), 0, s, in, ws, N, pe);
    else hipLaunchKernelGGL((pack_kernel<PLANES, DIR, false>), grid, dim3(256), 0, s, in, ws, N, pe);
    return hipGetLastError();
}

Params make_params(int planes, const void* ws, void* out, bool out_c128, int N, int batch, double scale) {
    return Params{ws, out, N, out_c128 ? 1 : 0, scale,
                  planes == 2 ? prescale_exponents(const_cast<void*>(ws), N, batch) : nullptr};
}

}  // namespace

int mfma_tile_count(int /*planes*/) { return NTILES; }

bool mfma_tile_valid(int planes, int tile, int N) {
    if (tile < 1 || tile > NTILES) return false;
    const TileDesc t = TILES[tile - 1];
    if (!t.lds && !ring_tile_ok(planes, t.rb)) return false;
    return padded_dim(N) >= (uint32_t)(t.rb * t.waves * 32);
}

int mfma_default_tile(int planes, int N) {
    if (planes == 1 && N >= 8) return 15;   // LDS-staged, 256 rows: fastest binary32 shape
    if (N >= 9) return 1;
    if (N == 8) return 3;
    if (N == 7) return 6;
    if (N == 6) return 9;
    return 5;
}

bool mfma_tile_valid_hermitian(int planes, int tile, int N) {
    return mfma_tile_valid(planes, tile, N) && !TILES[tile - 1].lds;
}

int mfma_default_tile_hermitian(int planes, int N) {
    if (planes == 1 && N >= 8) return 3;    // 2 x 32 rows per wave, 4 waves (register ring)
    // One wave of 4 x 32 rows per workgroup: row-halved pairs from X0 >= 128
    // on, and the doubled epilogue of one workgroup overlaps the others'
    // contraction (N = 12-14: 4-13% faster than tile 1).
    if (planes >= 2 && N >= 12) return 7;
    return mfma_default_tile(planes, N);
}

size_t mfma_workspace_bytes(int planes, int N, int batch) {
    size_t b = packed_bytes(planes, N, batch);
    if (planes == 2)
        b += round256(sizeof(int) * (size_t)batch) + sizeof(float) * (size_t)absmax_blocks(N) * (size_t)batch;
    return b;
}

hipError_t launch_mfma_pack(Dir dir, int planes, const void* in, bool in_c128, int N, int batch, void* ws,
                            hipStream_t stream) {
    if (planes == 3)
        return dir == FORWARD ? launch_pack<3, FORWARD>(in, in_c128, ws, N, batch, stream)
                              : launch_pack<3, ADJOINT>(in, in_c128, ws, N, batch, stream);
    if (planes == 2)
        return dir == FORWARD ? launch_pack<2, FORWARD>(in, in_c128, ws, N, batch, stream)
                              : launch_pack<2, ADJOINT>(in, in_c128, ws, N, batch, stream);
    return dir == FORWARD ? launch_pack<1, FORWARD>(in, in_c128, ws, N, batch, stream)
                          : launch_pack<1, ADJOINT>(in, in_c128, ws, N, batch, stream);
}

hipError_t launch_mfma_contract(Dir dir, int planes, const void* ws, void* out, bool out_c128, int N, int batch,
                                double scale, int tile, hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile(planes, N);
    if (!mfma_tile_valid(planes, tile, N)) return hipErrorInvalidValue;
    const Params p = make_params(planes, ws, out, out_c128, N, batch, scale);
    if (planes == 3)
        return dir == FORWARD ? launch_tile<3, FORWARD>(tile, p, batch, stream)
                              : launch_tile<3, ADJOINT>(tile, p, batch, stream);
    if (planes == 2)
        return dir == FORWARD ? launch_tile<2, FORWARD>(tile, p, batch, stream)
                              : launch_tile<2, ADJOINT>(tile, p, batch, stream);
    return dir == FORWARD ? launch_tile<1, FORWARD>(tile, p, batch, stream)
                          : launch_tile<1, ADJOINT>(tile, p, batch, stream);
}

hipError_t launch_mfma(Dir dir, int planes, const void* in, bool in_c128, void* out,
                       bool out_c128, int N, int batch, double scale, int tile, void* ws,
                       hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile(planes, N);
    if (!mfma_tile_valid(planes, tile, N)) return hipErrorInvalidValue;
    const hipError_t e = launch_mfma_pack(dir, planes, in, in_c128, N, batch, ws, stream);
    if (e != hipSuccess) return e;
    return launch_mfma_contract(dir, planes, ws, out, out_c128, N, batch, scale, tile, stream);
}

hipError_t launch_mfma_contract_hermitian(int planes, const void* ws, void* out, bool out_c128, int N, int batch,
                                          double scale, int tile, hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile_hermitian(planes, N);
    if (!mfma_tile_valid_hermitian(planes, tile, N)) return hipErrorInvalidValue;
    const Params p = make_params(planes, ws, out, out_c128, N, batch, scale);
    if (planes == 3) return launch_tile<3, FORWARD, true>(tile, p, batch, stream);
    if (planes == 2) return launch_tile<2, FORWARD, true>(tile, p, batch, stream);
    return launch_tile<1, FORWARD, true>(tile, p, batch, stream);
}

// The pack skips only what no Hermitian tile reads: from the largest
// half-walk threshold of any register-ring tile on, so that the pack does not
// depend on the contraction's tile choice.
uint32_t herm_pack_min(int planes) {
    uint32_t h = 128u;
    for (int k = 0; k < NTILES; ++k) {
        const TileDesc t = TILES[k];
        if (t.lds || !ring_tile_ok(planes, t.rb)) continue;
        const uint32_t v = herm_half_from(planes, t.rb, t.pf);
        if (v > h) h = v;
    }
    return h;
}

hipError_t launch_mfma_pack_hermitian(int planes, const void* in, bool in_c128, int N, int batch, void* ws,
                                      hipStream_t stream) {
    const uint32_t hmin = herm_pack_min(planes);
    if (hmin < 128u || (hmin & (hmin - 1u))) return hipErrorInvalidValue;   // the grid mapping needs both
    const dim3 grid(herm_pack_tiles(N, hmin), batch);
    const int* pe = nullptr;
    if (planes == 3) {
        if (in_c128) hipLaunchKernelGGL((pack_herm_kernel<3, true>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
        else hipLaunchKernelGGL((pack_herm_kernel<3, false>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
    } else if (planes == 2) {
        const hipError_t e = launch_prescale_hermitian(in, in_c128, ws, N, batch, stream);
        if (e != hipSuccess) return e;
        pe = prescale_exponents(ws, N, batch);
        if (in_c128) hipLaunchKernelGGL((pack_herm_kernel<2, true>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
        else hipLaunchKernelGGL((pack_herm_kernel<2, false>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
    } else {
        if (in_c128) hipLaunchKernelGGL((pack_herm_kernel<1, true>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
        else hipLaunchKernelGGL((pack_herm_kernel<1, false>), grid, dim3(256), 0, stream, in, ws, N, hmin, pe);
    }
    return hipGetLastError();
}

hipError_t launch_mfma_hermitian(int planes, const void* in, bool in_c128, void* out, bool out_c128, int N,
                                 int batch, double scale, int tile, void* ws, hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile_hermitian(planes, N);
    if (!mfma_tile_valid_hermitian(planes, tile, N)) return hipErrorInvalidValue;
    const hipError_t e = launch_mfma_pack_hermitian(planes, in, in_c128, N, batch, ws, stream);
    if (e != hipSuccess) return e;
    return launch_mfma_contract_hermitian(planes, ws, out, out_c128, N, batch, scale, tile, stream);
}


}  // namespace pauli