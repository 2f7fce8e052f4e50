// Single-matrix entry of the matrix-core path (see mfma_tile.hpp for the
// method): one pack launch over all pack tiles of the batch of equal-order
// matrices, then one contraction launch over all output tiles.
#include "mfma_tile.hpp"

namespace pauli {
namespace {

using namespace mfma;

template <int PLANES, int DIR, bool IN128>
__global__ __launch_bounds__(256) void pack_kernel(const void* __restrict__ in, void* __restrict__ ws, int N) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[pack_lds_bytes<PLANES, DIR>()];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    pack_tile<PLANES, DIR, IN128>(src, wsm, N, blockIdx.x, lds);
}

// Pack for the Hermitian contraction: the K ranges its half walk skips are not packed.
template <int PLANES, bool IN128>
__global__ __launch_bounds__(256) void pack_herm_kernel(const void* __restrict__ in, void* __restrict__ ws, int N,
                                                        uint32_t hmin) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[pack_lds_bytes<PLANES>()];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * Dp * Dp * Pack<PLANES>::EB;
    pack_tile<PLANES, FORWARD, IN128>(src, wsm, N, herm_pack_tile(N, hmin, blockIdx.x), lds);
}

struct Params {
    const void* ws;
    void* out;
    int N;
    int out128;
    double scale;
};

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
    contract_tile<PLANES, RB, WAVES, DIR, PF, HERM>(wsm, dst, prm.N, xb, L % nMB, prm.scale, prm.out128, lds);
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
    contract_tile_lds<PLANES, RB, DIR, AHEAD>(wsm, dst, prm.N, L / nMB, L % nMB, prm.scale, prm.out128, lds);
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
        const int lds = WAVES * 1024 * (p.out128 ? 16 : 8);
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

template <int PLANES, int DIR>
hipError_t launch_pack(const void* in, bool in128, void* ws, int N, int batch, hipStream_t s) {
    const dim3 grid(pack_tiles(N), batch);
    if (in128) hipLaunchKernelGGL((pack_kernel<PLANES, DIR, true>), grid, dim3(256), 0, s, in, ws, N);
    else hipLaunchKernelGGL((pack_kernel<PLANES, DIR, false>), grid, dim3(256), 0, s, in, ws, N);
    return hipGetLastError();
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
    return mfma_default_tile(planes, N);
}

size_t mfma_workspace_bytes(int planes, int N, int batch) {
    const size_t Dp = padded_dim(N);
    return Dp * Dp * (size_t)(planes == 3 ? Pack<3>::EB : Pack<1>::EB) * (size_t)batch;
}

hipError_t launch_mfma_pack(Dir dir, int planes, const void* in, bool in_c128, int N, int batch, void* ws,
                            hipStream_t stream) {
    if (planes == 3)
        return dir == FORWARD ? launch_pack<3, FORWARD>(in, in_c128, ws, N, batch, stream)
                              : launch_pack<3, ADJOINT>(in, in_c128, ws, N, batch, stream);
    return dir == FORWARD ? launch_pack<1, FORWARD>(in, in_c128, ws, N, batch, stream)
                          : launch_pack<1, ADJOINT>(in, in_c128, ws, N, batch, stream);
}

hipError_t launch_mfma_contract(Dir dir, int planes, const void* ws, void* out, bool out_c128, int N, int batch,
                                double scale, int tile, hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile(planes, N);
    if (!mfma_tile_valid(planes, tile, N)) return hipErrorInvalidValue;
    Params p{ws, out, N, out_c128 ? 1 : 0, scale};
    if (planes == 3)
        return dir == FORWARD ? launch_tile<3, FORWARD>(tile, p, batch, stream)
                              : launch_tile<3, ADJOINT>(tile, p, batch, stream);
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
    Params p{ws, out, N, out_c128 ? 1 : 0, scale};
    return planes == 3 ? launch_tile<3, FORWARD, true>(tile, p, batch, stream)
                       : launch_tile<1, FORWARD, true>(tile, p, batch, stream);
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
    if (planes == 3) {
        if (in_c128) hipLaunchKernelGGL((pack_herm_kernel<3, true>), grid, dim3(256), 0, stream, in, ws, N, hmin);
        else hipLaunchKernelGGL((pack_herm_kernel<3, false>), grid, dim3(256), 0, stream, in, ws, N, hmin);
    } else {
        if (in_c128) hipLaunchKernelGGL((pack_herm_kernel<1, true>), grid, dim3(256), 0, stream, in, ws, N, hmin);
        else hipLaunchKernelGGL((pack_herm_kernel<1, false>), grid, dim3(256), 0, stream, in, ws, N, hmin);
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