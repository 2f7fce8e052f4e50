// All 4^N coefficients by fast Walsh-Hadamard transforms, O(N 4^N), in
// binary64 -- not the paper's O(8^N) evaluation but the same result: for
// every flip mask x the coefficients c(x, .) are the Sylvester-Hadamard
// transform of the gathered diagonal v_x[i] = G[i^x][i] followed by the
// phase (-i)^{popc(x&z)} and 2^-N (T. Jones 2024, section 2,
// Eq. (c_def_in_terms_of_fn) with the Pauli matrices of Eq. (3)).
//
// With i = 32 i_h + i_l and z = 32 z_h + z_l the sign (-1)^{popc(i&z)}
// factors into (-1)^{popc(i_l&z_l)} (-1)^{popc(i_h&z_h)}, so the transform
// splits into two HBM passes through a binary64 intermediate
//   U[x][z_l][i_h] = sum_{i_l} (-1)^{popc(i_l&z_l)} G[(32 i_h + i_l)^x][32 i_h + i_l]
//   c(x, 32 z_h + z_l) = 2^-N (-i)^{popc(x&z)} sum_{i_h} (-1)^{popc(i_h&z_h)} U[x][z_l][i_h]
// (U holds 4^N complex binary64 values, 16 bytes each, in the workspace).
//
// Pass 1: a workgroup owns 32 flip masks x0..x0+31 and 8 consecutive i_h.
// For each i_h the 32 x 32 block of G at rows (32 i_h ^ x0) .. +31, columns
// 32 i_h .. +31 holds exactly the 32 diagonals' entries for those i (entry
// (r, c) belongs to x_l = r ^ c, i_l = c), so it is loaded whole, widened to
// binary64 in LDS, and read back transposed: thread t takes x_l = t >> 3 and
// i_l = 4 (t & 7) + k, k < 4.  The 32-point butterflies run over k inside the
// thread and over lanes t ^ 1, t ^ 2, t ^ 4 (i_l bits 2..4).  The 8 values
// of each (x, z_l) for the workgroup's 8 i_h are one 128-byte run of U.
//
// Pass 2: a workgroup owns 16 vectors U[x][z_l][.] -- 4 flip masks x_l =
// 4a..4a+3 and 4 phase values z_l = 4b..4b+3 of one 32-mask block -- with
// 16 threads per vector holding i_h = q + 16 k.  Butterflies run over k in
// the thread and over lanes q ^ 1, 2, 4, 8.  For each z_h the 16 results are
// the 16 consecutive coefficients n with fixed high bits (n's low four bits
// are (x^z)_0, z_0, (x^z)_1, z_1), so they are staged in LDS and stored as one
// contiguous 128-byte (complex64) or 256-byte (complex128) run.
#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace {

constexpr int HB = 8;                   // i_h values per pass-1 workgroup

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ inline double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ inline double2 shfl_xor2(double2 v, int m) {
    return make_double2(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

// Butterfly across lanes on index bit owned by lane mask m: the lane whose
// m-bit is clear keeps a + b, its partner keeps a - b.
__device__ inline double2 lane_butterfly(double2 v, int lane, int m) {
    const double2 p = shfl_xor2(v, m);
    return (lane & m) ? sub2(p, v) : add2(v, p);
}

template <bool IN128>
__device__ inline double2 load_g(const void* G, size_t idx) {
    if constexpr (IN128) {
        return ((const double2*)G)[idx];
    } else {
        const float2 g = ((const float2*)G)[idx];
        return make_double2((double)g.x, (double)g.y);
    }
}

template <bool IN128>
__global__ __launch_bounds__(256) void fwht_pass1(const void* __restrict__ Gall, double2* __restrict__ Uall, int N) {
    __shared__ double2 tile[32 * 33];    // [row][column], padded row
    const uint32_t D = 1u << N, M = D >> 5;
    const uint32_t x0 = blockIdx.x * 32u, h0 = blockIdx.y * HB;
    const size_t mat = (size_t)D * D;
    const unsigned char* G = (const unsigned char*)Gall + (size_t)blockIdx.z * mat * (IN128 ? 16 : 8);
    double2* U = Uall + (size_t)blockIdx.z * mat;
    const int t = threadIdx.x, lane = t & 63;
    const int lr = t >> 3, lc = (t & 7) * 4;       // load: row, first column of 4
    const int xl = t >> 3, il0 = (t & 7) * 4;      // transform: flip mask, first i_l of 4

    double2 acc[4][HB];
#pragma unroll
    for (int h = 0; h < HB; ++h) {
        const uint32_t ih = h0 + h;
        const uint32_t row = ((ih << 5) ^ x0) + lr, col = (ih << 5) + lc;
        double2 g[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = load_g<IN128>(G, (size_t)row * D + col + k);
        if (h > 0) __syncthreads();              // previous tile fully read
#pragma unroll
        for (int k = 0; k < 4; ++k) tile[lr * 33 + lc + k] = g[k];
        __syncthreads();
        double2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int il = il0 + k;
            v[k] = tile[(il ^ xl) * 33 + il];
        }
        // i_l bits 0 and 1: inside the thread
        {
            const double2 a0 = add2(v[0], v[1]), a1 = sub2(v[0], v[1]);
            const double2 a2 = add2(v[2], v[3]), a3 = sub2(v[2], v[3]);
            v[0] = add2(a0, a2);
            v[2] = sub2(a0, a2);
            v[1] = add2(a1, a3);
            v[3] = sub2(a1, a3);
        }
        // i_l bits 2, 3, 4: lanes t ^ 1, t ^ 2, t ^ 4
#pragma unroll
        for (int m = 1; m <= 4; m <<= 1)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = lane_butterfly(v[k], lane, m);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k][h] = v[k];
    }
    // U[x][z_l][h0 .. h0 + 7]: one contiguous 128-byte run per (x, z_l)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t zl = il0 + k;
        double2* dst = U + ((size_t)(x0 + xl) * 32u + zl) * M + h0;
#pragma unroll
        for (int h = 0; h < HB; ++h) dst[h] = acc[k][h];
    }
}

// EPT = M / 16 elements per thread (M = 2^(N-5) values of i_h per vector).
template <int EPT, bool OUT128>
__global__ __launch_bounds__(256) void fwht_pass2(const double2* __restrict__ Uall, void* __restrict__ outall, int N,
                                                  double scale) {
    extern __shared__ __attribute__((aligned(16))) unsigned char stage[];   // [z_h][16] coefficients
    constexpr uint32_t M = 16u * EPT;
    constexpr int ESZ = OUT128 ? 16 : 8;
    const uint32_t D = 1u << N;
    const size_t mat = (size_t)D * D;
    const uint32_t x0 = blockIdx.x * 32u;
    const uint32_t a = blockIdx.y & 7u, b = blockIdx.y >> 3;      // x_l quad, z_l quad
    const double2* U = Uall + (size_t)blockIdx.z * mat;
    unsigned char* out = (unsigned char*)outall + (size_t)blockIdx.z * mat * ESZ;
    const int t = threadIdx.x, lane = t & 63;
    const int vec = t >> 4, q = t & 15;
    const uint32_t xl = 4u * a + (uint32_t)(vec & 3), zl = 4u * b + (uint32_t)(vec >> 2);
    const uint32_t x = x0 + xl;

    double2 v[EPT];
    const double2* src = U + ((size_t)x * 32u + zl) * M + q;
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = src[16 * k];

    // i_h bits 4 .. log2(M)-1: over k inside the thread
#pragma unroll
    for (int s = 1; s < EPT; s <<= 1)
#pragma unroll
        for (int k = 0; k < EPT; ++k)
            if ((k & s) == 0) {
                const double2 p = v[k], r = v[k + s];
                v[k] = add2(p, r);
                v[k + s] = sub2(p, r);
            }
    // i_h bits 0 .. 3: lanes q ^ 1, 2, 4, 8
#pragma unroll
    for (int m = 1; m <= 8; m <<= 1)
#pragma unroll
        for (int k = 0; k < EPT; ++k) v[k] = lane_butterfly(v[k], lane, m);

    // phase, scale, stage: slot = (x^z)_0 | z_0 << 1 | (x^z)_1 << 2 | z_1 << 3
    const uint32_t slot = ((xl ^ zl) & 1u) | ((zl & 1u) << 1) | (((xl ^ zl) & 2u) << 1) | ((zl & 2u) << 2);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t zh = (uint32_t)q + 16u * k;
        const uint32_t z = (zh << 5) + zl;
        double re = v[k].x * scale, im = v[k].y * scale;
        rotate_minus_i(re, im, (uint32_t)__popc(x & z));
        unsigned char* dstl = stage + ((size_t)zh * 16u + slot) * ESZ;
        if constexpr (OUT128) *(double2*)dstl = make_double2(re, im);
        else *(float2*)dstl = make_float2((float)re, (float)im);
    }
    __syncthreads();
    // M runs of 16 coefficients (16 * ESZ bytes each), 16-byte stores
    constexpr uint32_t CH = (16u * ESZ) / 16u;    // 16-byte chunks per run
    const uint32_t xb4 = x0 + 4u * a, zb4 = 4u * b;
    for (uint32_t j = (uint32_t)t; j < M * CH; j += 256u) {
        const uint32_t zh = j / CH, part = j % CH;
        const uint32_t base = pauli_index(xb4, (zh << 5) + zb4);   // low four bits are zero
        *(u32x4_t*)(out + (size_t)base * ESZ + part * 16u) = *(const u32x4_t*)(stage + ((size_t)zh * CH + part) * 16u);
    }
}

template <int EPT>
hipError_t launch_pass2(const double2* U, void* out, bool out128, int N, int batch, hipStream_t s) {
    const uint32_t D = 1u << N;
    const dim3 grid(D / 32u, 64u, (uint32_t)batch);
    const size_t lds = (size_t)16u * EPT * 16u * (out128 ? 16u : 8u);
    const double scale = 1.0 / (double)D;
    hipError_t e;
    if (out128) {
        e = hipFuncSetAttribute((const void*)fwht_pass2<EPT, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_pass2<EPT, true>), grid, dim3(256), lds, s, U, out, N, scale);
    } else {
        e = hipFuncSetAttribute((const void*)fwht_pass2<EPT, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_pass2<EPT, false>), grid, dim3(256), lds, s, U, out, N, scale);
    }
    return hipGetLastError();
}

}  // namespace

bool fwht_supported(int N) { return N >= FWHT_N_MIN && N <= FWHT_N_MAX; }

size_t fwht_workspace_bytes(int N, int batch) {
    return ((size_t)1 << (2 * N)) * 16u * (size_t)batch;
}

hipError_t launch_fwht(const void* G, bool in_c128, void* out, bool out_c128, int N, int batch, void* ws,
                       hipStream_t s) {
    if (!fwht_supported(N)) return hipErrorInvalidValue;
    const uint32_t D = 1u << N, M = D >> 5;
    double2* U = (double2*)ws;
    const dim3 g1(D / 32u, M / HB, (uint32_t)batch);
    if (in_c128) hipLaunchKernelGGL(fwht_pass1<true>, g1, dim3(256), 0, s, G, U, N);
    else hipLaunchKernelGGL(fwht_pass1<false>, g1, dim3(256), 0, s, G, U, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (N) {
        case 9: return launch_pass2<1>(U, out, out_c128, N, batch, s);
        case 10: return launch_pass2<2>(U, out, out_c128, N, batch, s);
        case 11: return launch_pass2<4>(U, out, out_c128, N, batch, s);
        case 12: return launch_pass2<8>(U, out, out_c128, N, batch, s);
        case 13: return launch_pass2<16>(U, out, out_c128, N, batch, s);
        case 14: return launch_pass2<32>(U, out, out_c128, N, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pauli
