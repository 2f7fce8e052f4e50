// Fixed-point int8 variant of the matrix-core contraction (gfx950).
//
// The same dense contraction as the split paths (mfma_tile.hpp),
//
//     C[z][x] = sum_i H[z][i] v_x[i],   H[z][i] = (-1)^{popc(i & z)},
//     c(x, z) = 2^-N (-i)^{popc(x&z)} C[z][x]        (Eq. (c_def_in_terms_of_fn)),
//
// with G turned into integers and the integers into three int8 digit planes.
// A +-1 times int8 product summed by the int8 matrix cores is exact in
// int32, so the contraction itself rounds nothing: the only errors are the
// quantisation of G and the rounding of the final scaling.
//
// Quantisation, per matrix: m = the largest |Re g|, |Im g| (in the input's
// precision), e its binary exponent (m = mm 2^e, 1 <= mm < 2), and
// L = 8355711 = 127 (2^16 + 2^8 + 1); each component becomes
//     q = rint(g 2^-e s),   s = L / mm,   |q| <= L,
// and q = 65536 d2 + 256 d1 + d0 with balanced base-256 digits d0, d1 in
// [-128, 127] and |d2| <= 127 (L is the largest bound for which the top
// digit stays within int8).  |g - q mm 2^e / L| <= mm 2^e / (2 L), so each
// coefficient is off by at most 2^-N sum_i |err_i| <= m / (2 L) (about
// 6e-8 m) per component, whatever N; independent roundings make the
// typical error smaller by about 2^(-N/2).  The bound is relative to the
// largest entry of G, not to each entry: fixed point, unlike the
// floating-point splits.
//
// Sums: A_d = sum_i H[z][i] d_i per digit plane, |A_d| <= 128 2^N.  The
// contraction walks K twice: pass 1 with the d2 and d1 planes into two int32
// accumulator sets, folded into h = 256 A2 + A1 (|h| < 2^31 for N <= 16
// because |d2| <= 127), pass 2 with the d0 plane; the epilogue forms
// 256 h + A0 = sum_i H[z][i] q_i exactly in binary64 and scales it by
// 2^(e-N) mm / L.  Two passes keep two accumulator sets live instead of
// three, so the 4 x 32-row tiles fit the register file.
//
// Kernels, launched in order on one stream (every value a kernel reads was
// written by an earlier one, so the workspace needs no clearing):
//   i8_absmax_kernel   partial maxima of |Re g|, |Im g| over R ranges
//                      (i8_absmax_lower_kernel: the lower triangle of a
//                      Hermitian matrix)
//   i8_scale_kernel    one scale record per matrix
//   i8_pack_kernel     gather + quantise + digit split into fragments
//   i8_contract_kernel the two walks over K and the epilogue (HERM: the
//                      Hermitian shortcut, a quarter of the walks)
#include "mfma_tile.hpp"

namespace pauli {
namespace {

using namespace mfma;

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr double I8_LIMIT = 8355711.0;   // 127 * (65536 + 256 + 1)
constexpr int I8_NPL = 6;                // fragments per slice: 3 digit planes x (re, im)
constexpr int I8_SK = 32;                // K values per slice (one 32x32x32 MFMA)
constexpr int I8_SLICE = I8_NPL * FRAG;  // bytes per slice of one 32-mask slab
constexpr int I8_RB = 4;                 // 4 x 32 rows per wave, 32 flip masks
// Waves per workgroup: 4 for the general contraction; 1 for the Hermitian
// one, whose doubled epilogue then overlaps other workgroups' walks instead
// of holding three more waves at its barriers (measured 2-5% faster there,
// 1% slower for the general one).
constexpr int i8_waves(bool herm) { return herm ? 1 : 4; }
constexpr int i8_rows(bool herm) { return i8_waves(herm) * I8_RB * 32; }
constexpr int I8_PF1 = 4, I8_PF2 = 8;    // ring depth (slices) of the two passes
constexpr int I8_STEP = 16;              // slices per unrolled step (8 when a slab has only 8)
// Hermitian input: slabs of flip masks X0 >= I8_HERM_FROM walk half of K and
// compute half of the rows (see i8_contract_kernel).  A power of two >= 128
// (the pack's K tile), >= 32 * I8_STEP (a step's slices never straddle the
// skipped bit) and >= the rows of a workgroup (the skipped row bit spans
// whole workgroup tiles).
constexpr uint32_t I8_HERM_FROM = 512;

// Scale record of one matrix (see the header comment): q = rint(ldexp(g, -e) * s),
// value = ldexp(sum * r, e) with r = mm / L times the caller's scale.
struct I8Scale {
    double s;   // L / mm (0 for an all-zero or non-finite matrix)
    double r;   // mm / L (NaN for a non-finite matrix, 0 for an all-zero one)
    int e;
    int pad[3];
};

__host__ __device__ inline size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Reduction blocks per matrix: a power of two dividing 4^N, one per 4096
// elements, at most 1024.
__host__ __device__ inline uint32_t i8_absmax_blocks(int N) {
    const int lg = 2 * N - 12;
    return lg <= 0 ? 1u : (lg >= 10 ? 1024u : 1u << lg);
}

__host__ __device__ inline size_t i8_packed_bytes(int N) {
    const size_t Dp = padded_dim(N);
    return Dp * Dp * I8_NPL;
}

// Workspace: [packed operands | scale records | partial maxima].
I8Scale* i8_scales(void* ws, int N, int batch) {
    return (I8Scale*)((unsigned char*)ws + round256(i8_packed_bytes(N) * (size_t)batch));
}
double* i8_partials(void* ws, int N, int batch) {
    return (double*)((unsigned char*)i8_scales(ws, N, batch) + round256(sizeof(I8Scale) * (size_t)batch));
}

// Largest of m over a 256-thread workgroup; every thread gets it.
__device__ inline double block_max256_f64(double m, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    return __builtin_fmax(__builtin_fmax(red[0], red[1]), __builtin_fmax(red[2], red[3]));
}

// |a| as the running maximum sees it: +inf for a NaN or infinite component,
// so that any non-finite input reaches the scale record.
__device__ inline double mag(double a) {
    const double v = __builtin_fabs(a);
    return v <= 1.7976931348623157e308 ? v : __builtin_inf();
}

template <bool IN128>
__global__ __launch_bounds__(256) void i8_absmax_kernel(const void* __restrict__ in, int N,
                                                        double* __restrict__ partial, uint32_t R) {
    __shared__ double red[4];
    const size_t n = (size_t)1 << (2 * N);
    const size_t per = n / R;
    const size_t lo = (size_t)blockIdx.x * per;
    double m = 0.0;
    if constexpr (IN128) {
        const double2* p = (const double2*)in + (size_t)blockIdx.y * n + lo;
        for (size_t i = threadIdx.x; i < per; i += 256) {
            const double2 v = p[i];
            m = __builtin_fmax(m, __builtin_fmax(mag(v.x), mag(v.y)));
        }
    } else if (per % 2 == 0) {
        const float4* p = (const float4*)((const float2*)in + (size_t)blockIdx.y * n + lo);
        for (size_t i = threadIdx.x; i < per / 2; i += 256) {
            const float4 v = p[i];
            m = __builtin_fmax(m, __builtin_fmax(__builtin_fmax(mag(v.x), mag(v.y)),
                                                 __builtin_fmax(mag(v.z), mag(v.w))));
        }
    } else {
        const float2* p = (const float2*)in + (size_t)blockIdx.y * n + lo;
        for (size_t i = threadIdx.x; i < per; i += 256) {
            const float2 v = p[i];
            m = __builtin_fmax(m, __builtin_fmax(mag(v.x), mag(v.y)));
        }
    }
    m = block_max256_f64(m, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * R + blockIdx.x] = m;
}

// The same reduction over the lower triangle of a Hermitian matrix (whose
// upper triangle repeats it with the imaginary parts negated): workgroup
// blockIdx.x takes row pairs r, D-1-r (r + 1 and D - r elements of the
// triangle, D + 1 together), so R = min(i8_absmax_blocks(N), D / 2)
// workgroups read half of G.  D >= 2.
template <bool IN128>
__global__ __launch_bounds__(256) void i8_absmax_lower_kernel(const void* __restrict__ in, int N,
                                                              double* __restrict__ partial, uint32_t R) {
    __shared__ double red[4];
    const uint32_t D = 1u << N;
    const uint32_t ppb = (D / 2u) / R;   // row pairs per workgroup
    const size_t mat = (size_t)D * D;
    double m = 0.0;
    for (uint32_t pp = 0; pp < ppb; ++pp) {
        const uint32_t r = blockIdx.x * ppb + pp;
        for (uint32_t e = threadIdx.x; e <= D; e += 256) {
            const size_t idx = e <= r ? (size_t)r * D + e : (size_t)(D - 1u - r) * D + (e - r - 1u);
            if constexpr (IN128) {
                const double2 v = ((const double2*)in)[(size_t)blockIdx.y * mat + idx];
                m = __builtin_fmax(m, __builtin_fmax(mag(v.x), mag(v.y)));
            } else {
                const float2 v = ((const float2*)in)[(size_t)blockIdx.y * mat + idx];
                m = __builtin_fmax(m, __builtin_fmax(mag(v.x), mag(v.y)));
            }
        }
    }
    m = block_max256_f64(m, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * R + blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void i8_scale_kernel(const double* __restrict__ partial, uint32_t R,
                                                       I8Scale* __restrict__ rec) {
    __shared__ double red[4];
    double m = 0.0;
    for (uint32_t i = threadIdx.x; i < R; i += 256) m = __builtin_fmax(m, partial[(size_t)blockIdx.x * R + i]);
    m = block_max256_f64(m, red);
    if (threadIdx.x == 0) {
        I8Scale q = {0.0, 0.0, 0, {0, 0, 0}};
        if (!(m <= 1.7976931348623157e308)) {
            q.r = __builtin_nan("");        // non-finite input: every coefficient NaN
        } else if (m > 0.0) {
            int e;
            const double mm = 2.0 * __builtin_frexp(m, &e);   // m = mm 2^(e-1), mm in [1, 2)
            e -= 1;
            q.s = I8_LIMIT / mm;
            q.r = mm / I8_LIMIT;
            q.e = e;
        }
        rec[blockIdx.x] = q;
    }
}

// q of one component, as an int with |q| <= L.
__device__ inline int quantise(double g, double s, int e) {
    double t = __builtin_rint(__builtin_ldexp(g, -e) * s);
    t = __builtin_fmin(__builtin_fmax(t, -I8_LIMIT), I8_LIMIT);   // no-op for finite input; keeps NaN/inf in range
    return (int)t;
}

// Balanced base-256 digits of q (q = 65536 d2 + 256 d1 + d0): the byte of
// d0 is q mod 256, and q1 = (q - d0) / 256 = floor((q + 128) / 256).  Each
// byte lands at bit `sh` of its plane word.
__device__ inline void digits(int q, int sh, uint32_t& w2, uint32_t& w1, uint32_t& w0) {
    const int q1 = (q + 128) >> 8;
    const int q2 = (q1 + 128) >> 8;
    w0 |= ((uint32_t)q & 0xFFu) << sh;
    w1 |= ((uint32_t)q1 & 0xFFu) << sh;
    w2 |= ((uint32_t)q2 & 0xFFu) << sh;
}

// ---------------------------------------------------------------------------
// Packed operand, per matrix (Dp = max(2^N, 32)): fragment (xb, s, f) at
// ((xb * Dp/32 + s) * 6 + f) KiB, f = 2 * plane + (0 re, 1 im), plane 0 = d2,
// 1 = d1, 2 = d0; lane l = x_l + 32 h holds K = 32 s + 16 h + j, j < 16, of
// flip mask x = 32 xb + x_l, one byte each.
// ---------------------------------------------------------------------------
constexpr int I8_PITCH = PACK_KT + 16;   // LDS bytes per flip mask row of the staging tile

template <bool IN128>
__device__ inline double2 load_g(const unsigned char* base, size_t idx) {
    if constexpr (IN128) {
        return ((const double2*)base)[idx];
    } else {
        const float2 v = ((const float2*)base)[idx];
        return make_double2((double)v.x, (double)v.y);
    }
}

// Pack tile t of matrix blockIdx.y: 32 flip masks X0.. x KT values of i.  A
// thread gathers one aligned 4x4 micro-block of G (rows r0.., columns q0..),
// which the XOR map sends to 4 flip masks x 4 consecutive i, quantises it,
// and stores its digit bytes in the LDS staging tile; the workgroup then
// writes whole 1 KiB fragments.
// HERM: the grid holds only the tiles the Hermitian contraction's half walks
// read (herm_pack_tile with the threshold I8_HERM_FROM); the others are not
// packed.
template <bool IN128, bool HERM>
__global__ __launch_bounds__(256) void i8_pack_kernel(const void* __restrict__ in, void* __restrict__ ws, int N,
                                                      const I8Scale* __restrict__ rec) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[I8_NPL * XT * I8_PITCH];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    const uint32_t nKT = Dp / KT;
    const uint32_t t = HERM ? herm_pack_tile(N, I8_HERM_FROM, blockIdx.x) : blockIdx.x;
    const uint32_t xb = t / nKT, kt = t % nKT;
    const uint32_t X0 = xb * XT, Q0 = kt * KT;
    const bool full = D >= 32u;
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * i8_packed_bytes(N);
    const I8Scale sc = rec[blockIdx.y];
    const int tid = threadIdx.x;
    const int g = tid >> 6, w6 = tid & 63;   // 32x32 square g of the tile, micro-block w6 in it

    if ((uint32_t)tid < 2 * KT) {
        const int mr = w6 >> 3, mc = w6 & 7;
        const uint32_t q0 = Q0 + 32 * g + 4 * mc;                  // first column (= first i)
        const uint32_t r0 = (((Q0 + 32 * g) ^ X0) & ~31u) + 4 * mr;  // first row
        double2 v[16];
        if (!IN128 && full) {
            // complex64, D >= 32: each row's 4 elements are 32 aligned bytes, two 16-byte loads
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const float4* rp = (const float4*)(src + ((size_t)(r0 + a) * D + q0) * 8);
                const float4 u0 = rp[0], u1 = rp[1];
                v[a * 4 + 0] = make_double2((double)u0.x, (double)u0.y);
                v[a * 4 + 1] = make_double2((double)u0.z, (double)u0.w);
                v[a * 4 + 2] = make_double2((double)u1.x, (double)u1.y);
                v[a * 4 + 3] = make_double2((double)u1.z, (double)u1.w);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t r = r0 + a, q = q0 + b;
                    v[a * 4 + b] = (full || (r < D && q < D)) ? load_g<IN128>(src, (size_t)r * D + q) : make_double2(0.0, 0.0);
                }
        }
        // element (row r0 + a, column q0 + b) lies on flip mask (r0 ^ q0) + (a ^ b) at i = q0 + b
        const int xh = mr ^ mc;               // flip masks 4 xh .. 4 xh + 3 of the slab
        const int kh = 32 * g + 4 * mc;       // K slots kh .. kh + 3 of the tile
#pragma unroll
        for (int x2 = 0; x2 < 4; ++x2) {
            uint32_t w[6] = {0, 0, 0, 0, 0, 0};   // [2 * plane + comp]
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double2 e = v[((x2 ^ b) << 2) | b];   // row a = x2 ^ b, column b
                digits(quantise(e.x, sc.s, sc.e), 8 * b, w[0], w[2], w[4]);
                digits(quantise(e.y, sc.s, sc.e), 8 * b, w[1], w[3], w[5]);
            }
            unsigned char* row = lds + (xh * 4 + x2) * I8_PITCH + kh;
#pragma unroll
            for (int f = 0; f < 6; ++f) *(uint32_t*)(row + f * XT * I8_PITCH) = w[f];
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int xl = lane & 31, h = lane >> 5;
    const uint32_t nfrag = (KT / I8_SK) * I8_NPL;
    unsigned char* dst = wsm + ((size_t)xb * (Dp / I8_SK) + Q0 / I8_SK) * I8_SLICE;
    for (uint32_t f = wave; f < nfrag; f += 4) {
        const uint32_t s = f / I8_NPL, pl = f % I8_NPL;
        const unsigned char* p = lds + pl * XT * I8_PITCH + xl * I8_PITCH + s * I8_SK + h * 16;
        *(u32x4*)(dst + (size_t)f * FRAG + lane * 16) = *(const u32x4*)p;
    }
}

// Adjoint pack (reconstruction, gradient): the contraction input is
// In[z][x] = i^{popc(x&z)} c[n(x, z)], K = z.  The 32 x 32 coefficients of
// flip masks X0.. and phase masks zb = Q0 + 32 g .. are the 1024 consecutive
// entries from n(X0, zb); thread w6 takes 16 of them, o = 16 w6 + r with
// r = (x^z)_0 | z_0 << 1 | (x^z)_1 << 2 | z_1 << 3, i.e. 4 flip masks x 4
// consecutive z, applies the phase, quantises with the vector's scale record
// (the phase only permutes and negates components, so the largest component
// is the same) and stages the digits exactly as the forward pack does.
template <bool IN128>
__global__ __launch_bounds__(256) void i8_pack_adj_kernel(const void* __restrict__ in, void* __restrict__ ws, int N,
                                                          const I8Scale* __restrict__ rec) {
    // LDS: first each wave's 1024 coefficients (read lane-consecutive from
    // HBM, PADE elements of padding after every 16 so that the per-thread
    // reads of 16 consecutive entries fall in distinct banks), then, after a
    // barrier, the digit staging tile.
    constexpr int EW = IN128 ? 16 : 8;             // bytes per coefficient
    constexpr int PADE = IN128 ? 1 : 2;            // 16 bytes of padding per 16 coefficients
    constexpr int BLK = 1024 + 64 * PADE;          // elements per wave block
    constexpr int STAGE = I8_NPL * XT * I8_PITCH;
    constexpr int ADJB = 4 * BLK * EW;
    __shared__ __attribute__((aligned(16))) unsigned char lds[STAGE > ADJB ? STAGE : ADJB];
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    const uint32_t nKT = Dp / KT;
    const uint32_t t = blockIdx.x;
    const uint32_t xb = t / nKT, kt = t % nKT;
    const uint32_t X0 = xb * XT, Q0 = kt * KT;
    const bool full = D >= 32u;
    const unsigned char* src = (const unsigned char*)in + (size_t)blockIdx.y * D * D * (IN128 ? 16 : 8);
    unsigned char* wsm = (unsigned char*)ws + (size_t)blockIdx.y * i8_packed_bytes(N);
    const I8Scale sc = rec[blockIdx.y];
    const int tid = threadIdx.x;
    const int g = tid >> 6, w6 = tid & 63;
    const bool active = (uint32_t)tid < 2 * KT;
    const uint32_t zb = Q0 + 32 * g;
    const uint32_t nb = pauli_index(X0, zb);
    double2 v[16];

    if (full) {   // uniform
        unsigned char* blk = lds + g * BLK * EW;
        if (active) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t o = 64 * i + w6;
                const unsigned char* sp = src + (size_t)(nb + o) * EW;
                unsigned char* dp = blk + (o + PADE * (o >> 4)) * EW;
                if constexpr (IN128) *(double2*)dp = *(const double2*)sp;
                else *(float2*)dp = *(const float2*)sp;
            }
        }
        __syncthreads();
        if (active) {
            const unsigned char* mine = blk + w6 * (16 + PADE) * EW;   // entries 16 w6 .. 16 w6 + 15
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (IN128) {
                    v[2 * j] = ((const double2*)mine)[2 * j];
                    v[2 * j + 1] = ((const double2*)mine)[2 * j + 1];
                } else {
                    const float4 q = ((const float4*)mine)[j];
                    v[2 * j] = make_double2((double)q.x, (double)q.y);
                    v[2 * j + 1] = make_double2((double)q.z, (double)q.w);
                }
            }
        }
        __syncthreads();   // the staging below overwrites the LDS
    }

    if (active) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t o = 16 * w6 + r;
            const uint32_t zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
            const uint32_t z = zb + zl, x = X0 + xl;
            double2 c = full ? v[r] : make_double2(0.0, 0.0);
            if (!full && z < D && x < D) c = load_g<IN128>(src, nb + o);
            rotate_minus_i(c.x, c.y, 3u * (uint32_t)__popc(x & z));   // times i^{popc(x&z)}
            v[r] = c;
        }
        const uint32_t o = 16 * w6;
        const uint32_t zl0 = compact_even(o >> 1), xl0 = compact_even(o) ^ zl0;
        const int xh = (int)(xl0 >> 2);             // flip masks 4 xh .. 4 xh + 3 of the slab
        const int kh = 32 * g + (int)zl0;           // K slots (phase masks) kh .. kh + 3 of the tile
#pragma unroll
        for (int x2 = 0; x2 < 4; ++x2) {
            uint32_t w[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int d = x2 ^ b;   // (x ^ z) low bits for flip mask 4 xh + x2, phase mask kh + b
                const double2 e = v[(d & 1) | ((b & 1) << 1) | ((d >> 1) << 2) | ((b >> 1) << 3)];
                digits(quantise(e.x, sc.s, sc.e), 8 * b, w[0], w[2], w[4]);
                digits(quantise(e.y, sc.s, sc.e), 8 * b, w[1], w[3], w[5]);
            }
            unsigned char* row = lds + (xh * 4 + x2) * I8_PITCH + kh;
#pragma unroll
            for (int f = 0; f < 6; ++f) *(uint32_t*)(row + f * XT * I8_PITCH) = w[f];
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int xl = lane & 31, h = lane >> 5;
    const uint32_t nfrag = (KT / I8_SK) * I8_NPL;
    unsigned char* dst = wsm + ((size_t)xb * (Dp / I8_SK) + Q0 / I8_SK) * I8_SLICE;
    for (uint32_t f = wave; f < nfrag; f += 4) {
        const uint32_t s = f / I8_NPL, pl = f % I8_NPL;
        const unsigned char* p = lds + pl * XT * I8_PITCH + xl * I8_PITCH + s * I8_SK + h * 16;
        *(u32x4*)(dst + (size_t)f * FRAG + lane * 16) = *(const u32x4*)p;
    }
}

__device__ inline i32x16 mfma_i8(const i32x4& a, const i32x4& b, const i32x16& c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// This lane's +-1 fragment of the 32x32 Sylvester block: lane (row l32,
// half h), byte j = (-1)^{popc(l32 & (16 h + j))} as int8 (0x01 or 0xFF).
// Negation flips every byte between the two values (xor 0xFE).
__device__ inline i32x4 sign_fragment(int lane) {
    const uint32_t l32 = (uint32_t)lane & 31u, h = (uint32_t)lane >> 5;
    i32x4 A;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t q = 16u * h + 4u * (uint32_t)w + (uint32_t)b;
            word |= ((__popc(l32 & q) & 1) ? 0xFFu : 0x01u) << (8 * b);
        }
        A[w] = (int)word;
    }
    return A;
}

// One walk over the slices of the slab at `slab` with NP digit planes
// (P0, P0 + 1, ...) into acc[p][rb][cb].  The block of rows Pw + 32 rb
// against slice s (K block s) is the Sylvester block times
// (-1)^{popc((Pw/32 + rb) & s)}; Pw is a multiple of 128, so that sign is
// (-1)^{popc((Pw/32) & s)} (one per group of 4 slices) times
// (-1)^{popc(rb & s)} (fixed by s mod 4).  STEP slices per unrolled step;
// STEP = 1 (nS < 8, N < 8): one slice at a time with the signs evaluated at
// run time.  The walk visits nK slices: walk index c is slice
// ((c & ~low) << 1) | (c & low), all slices when low = ~0, and those with bit
// log2(low + 1) clear otherwise (a half walk; low + 1 >= STEP, so the slices
// of a step stay consecutive and aligned).  slab, nK, low and Pw are
// uniform; everything per lane is derived here from the thread index, so
// nothing of it stays live across the walks.
template <int NP, int P0, int PF, int STEP>
__device__ __attribute__((always_inline)) inline void walk(const unsigned char* __restrict__ slab, uint32_t nK,
                                                           uint32_t low, uint32_t Pw, i32x16 (&acc)[NP][I8_RB][2]) {
    constexpr int NF = 2 * NP;
    static_assert(STEP == 1 || (STEP % PF == 0 && STEP % 4 == 0), "ring and sign period nest in a step");
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const unsigned char* wsx = slab + lane * 16 + 2 * P0 * FRAG;
    const i32x4 Ap = sign_fragment(lane);
    const i32x4 An = Ap ^ (int)0xFEFEFEFE;
    const uint32_t pw5 = Pw >> 5;
    i32x4 ring[PF][NF];
    auto slice_of = [&](uint32_t c) { return ((c & ~low) << 1) | (c & low); };
    auto fetch = [&](int slot, uint32_t c) {
        const unsigned char* p = wsx + (size_t)slice_of(c) * I8_SLICE;
#pragma unroll
        for (int f = 0; f < NF; ++f) ring[slot][f] = *(const i32x4*)(p + f * FRAG);
    };
    if constexpr (STEP > 1) {
#pragma unroll
        for (int k = 0; k < PF; ++k) fetch(k, (uint32_t)k);
        // Wait for the prefetch once here: with these loads still in flight
        // at the loop head, the compiler's wait there (merging the prefetch
        // with the refills of the previous step) is a full drain of every
        // outstanding load, once per step; with them complete it waits only
        // for the slot the step starts with.
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt, lgkmcnt untouched
        for (uint32_t s0 = 0; s0 < nK; s0 += STEP) {
            const uint32_t sr = slice_of(s0);   // the step's slices are sr, sr + 1, ..., sr + STEP - 1
            i32x4 A0, A1;   // the group's sign applied: A0 for popc(rb & s) even, A1 odd
#pragma unroll
            for (int uu = 0; uu < STEP; ++uu) {
                const int slot = uu % PF;
                if (uu % 4 == 0) {
                    const bool gneg = __popc(pw5 & (sr + (uint32_t)uu)) & 1;
                    A0 = gneg ? An : Ap;
                    A1 = gneg ? Ap : An;
                }
#pragma unroll
                for (int rb = 0; rb < I8_RB; ++rb) {
                    const i32x4& A = (popc_const((uint32_t)rb & (uint32_t)(uu & 3)) & 1) ? A1 : A0;
#pragma unroll
                    for (int p = 0; p < NP; ++p)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb) acc[p][rb][cb] = mfma_i8(A, ring[slot][2 * p + cb], acc[p][rb][cb]);
                }
                // refill this slot PF slices ahead (the last refills reread the final slice, unused)
                __builtin_amdgcn_sched_barrier(0);
                const uint32_t nxt = s0 + (uint32_t)(uu + PF);
                fetch(slot, nxt < nK ? nxt : nK - 1);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        for (uint32_t c = 0; c < nK; ++c) {
            fetch(0, c);
            const uint32_t s = slice_of(c);
#pragma unroll
            for (int rb = 0; rb < I8_RB; ++rb) {
                const bool neg = __popc((pw5 + (uint32_t)rb) & s) & 1;
                const i32x4 A = neg ? An : Ap;
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) acc[p][rb][cb] = mfma_i8(A, ring[0][2 * p + cb], acc[p][rb][cb]);
            }
        }
    }
}

struct I8Params {
    const void* ws;
    void* out;
    int N;
    int out128;
    double scale;
    const I8Scale* rec;
};

// Output tile (slab xb, rows mb * MT ..) of matrix blockIdx.y, MT =
// i8_rows(HERM).  Waves whose rows lie beyond Dp (small N) skip the walks but
// take part in the epilogue barriers.  LDS: one 1024-coefficient stage per
// wave (two for HERM).
//
// HERM (Hermitian G): q(G[i][i ^ x]) = conj q(G[i ^ x][i]) exactly (the
// quantisation rounds symmetrically), so with b the top bit of X0 (set in
// every flip mask of the slab) the sum over the pair {i, i ^ x} is
// H[z][i] (v_i + (-1)^{popc(x&z)} conj v_i): twice the real part of the
// half sum T = sum over the i with bit b clear of H[z][i] v_i when
// popc(x&z) is even, 2i times its imaginary part when odd.  Slabs with
// X0 >= I8_HERM_FROM walk only those i, and since H[z][i] = H[z ^ 2^b][i]
// for them, rows z and z ^ 2^b have the same T with the parity flipped: the
// tile whose rows have bit b clear stores both (the partner's component in
// a second LDS stage) and the tile with it set does nothing.  Every sum is
// an exact integer, so the result equals the general kernel's bit for bit.
//
// ADJ (reconstruction, gradient): rows are i, K is z, and the sum for row i,
// column x is G[i ^ x][i] (times the caller's scale): the epilogue stages
// each 32 x 32 block as the aligned square of G it fills and stores it row
// by row.
template <int STEP, bool HERM, bool ADJ = false>
__global__ __launch_bounds__(256) void i8_contract_kernel(I8Params prm) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    constexpr int WAVES = i8_waves(HERM), MT = i8_rows(HERM);
    static_assert(!(HERM && ADJ), "the Hermitian shortcut is a forward-only property");
    static_assert(I8_HERM_FROM >= (uint32_t)MT && I8_HERM_FROM >= 32u * I8_STEP && I8_HERM_FROM >= (uint32_t)PACK_KT,
                  "threshold of the Hermitian half walk");
    const int N = prm.N;
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const uint32_t nMB = (Dp + MT - 1) / MT;
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    uint32_t xb = L / nMB;
    const uint32_t mb = L % nMB;
    if constexpr (HERM) {
        // The slabs below I8_HERM_FROM walk all of K for all rows (four times
        // the work of the others): deal slabs to the XCDs round-robin (XCD k,
        // which owns the logical range [k S, k S + S), gets slabs k, k + 8,
        // ...) so that those few spread over all eight.
        const uint32_t nXB = Dp / XT;
        if ((gridDim.x & 7u) == 0 && (nXB & 7u) == 0) {
            const uint32_t S = nXB >> 3;
            xb = (xb % S) * 8 + xb / S;
        }
    }
    const uint32_t X0 = xb * XT;
    const uint32_t nS = Dp / I8_SK;
    const unsigned char* slab =
        (const unsigned char*)prm.ws + (size_t)blockIdx.y * i8_packed_bytes(N) + (size_t)xb * nS * I8_SLICE;
    unsigned char* dst = (unsigned char*)prm.out + (size_t)blockIdx.y * D * D * (prm.out128 ? 16 : 8);
    const I8Scale sc = prm.rec[blockIdx.y];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t Pw = mb * MT + wave * I8_RB * 32;   // first row of this wave

    uint32_t nK = nS, low = ~0u, pair = 0;
    if constexpr (HERM) {
        if (X0 >= I8_HERM_FROM) {
            const uint32_t tb = 31u - (uint32_t)__builtin_clz(X0);   // bit b; 2^b >= MT
            low = (1u << (tb - 5u)) - 1u;                             // slice index bit b - 5 skipped
            nK = nS >> 1;
            pair = 1u << tb;
            if ((mb * (uint32_t)MT) & pair) return;   // the partner tile stores these rows
        }
    }

    // acc[0] ends as h (folded in place after pass 1), acc[1] as A0: the d0
    // accumulators reuse the d1 set, so two sets are live at any time.
    i32x16 acc[2][I8_RB][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int rb = 0; rb < I8_RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][rb][cb][r] = 0;
    if (Pw < Dp) {
        walk<2, 0, I8_PF1, STEP>(slab, nK, low, Pw, acc);
#pragma unroll
        for (int rb = 0; rb < I8_RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                acc[0][rb][cb] = acc[0][rb][cb] * 256 + acc[1][rb][cb];
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[1][rb][cb][r] = 0;
            }
        walk<1, 2, I8_PF2, STEP>(slab, nK, low, Pw, reinterpret_cast<i32x16(&)[1][I8_RB][2]>(acc[1]));
    }
    const auto& hi = acc[0];
    const i32x16(&lo)[1][I8_RB][2] = reinterpret_cast<const i32x16(&)[1][I8_RB][2]>(acc[1]);
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));   // the epilogue's lane values are formed here, not held across the walks
    const int lane = tid & 63;
    const int l32 = lane & 31, h = lane >> 5;

    // Epilogue: sum = 256 h + A0 exactly in binary64, times 2^(e-N) mm / L
    // (twice that after a half walk), the phase (-i)^{popc(x&z)}, staged so
    // the 32x32 block leaves as one contiguous run of coefficients starting
    // at n(X0, pb) (and, paired, at n(X0, pb ^ 2^b)).
    const double rs = sc.r * prm.scale * (pair ? 2.0 : 1.0);
    const int esz = prm.out128 ? 16 : 8;
    unsigned char* stage = lds + wave * 1024 * esz;
    unsigned char* stage2 = lds + (WAVES + wave) * 1024 * esz;   // HERM only
#pragma unroll
    for (int rb = 0; rb < I8_RB; ++rb) {
        const uint32_t pb = Pw + 32 * rb;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t pl = 8 * (r >> 2) + 4 * h + (r & 3);   // row of accumulator element r
            double re = __builtin_ldexp((256.0 * (double)hi[rb][0][r] + (double)lo[0][rb][0][r]) * rs, sc.e);
            double im = __builtin_ldexp((256.0 * (double)hi[rb][1][r] + (double)lo[0][rb][1][r]) * rs, sc.e);
            if constexpr (ADJ) {
                const uint32_t slot = ((pl ^ (uint32_t)l32) << 5) | pl;   // (row, col) inside the square
                if (prm.out128) *(double2*)(stage + slot * 16) = make_double2(re, im);
                else *(float2*)(stage + slot * 8) = make_float2((float)re, (float)im);
                continue;
            }
            const uint32_t ny = (uint32_t)__popc((X0 + l32) & (pb + pl));
            const uint32_t slot = pauli_index((uint32_t)l32, pl);
            if constexpr (HERM) {
                double qr = re, qi = im;   // row pb + pl ^ 2^b: the other component
                if (ny & 1) {
                    re = 0.0;
                    qi = 0.0;
                } else {
                    im = 0.0;
                    qr = 0.0;
                }
                if (pair) {
                    rotate_minus_i(qr, qi, ny + 1u);
                    if (prm.out128) *(double2*)(stage2 + slot * 16) = make_double2(qr, qi);
                    else *(float2*)(stage2 + slot * 8) = make_float2((float)qr, (float)qi);
                }
            }
            rotate_minus_i(re, im, ny);
            if (prm.out128) *(double2*)(stage + slot * 16) = make_double2(re, im);
            else *(float2*)(stage + slot * 8) = make_float2((float)re, (float)im);
        }
        __syncthreads();
        if constexpr (ADJ) {
            // 32x32 square of G: rows ((pb ^ X0) & ~31) + rl, columns pb + cl
            const uint32_t w = D < 32u ? D : 32u;
            const uint32_t rowbytes = w * esz;
            const uint32_t r0 = (pb ^ X0) & ~31u;
            if (pb < D) {
                if (rowbytes >= 16) {
                    for (uint32_t b = lane * 16; b < w * rowbytes; b += 64 * 16) {
                        const uint32_t rl = b / rowbytes, cb = b % rowbytes;
                        *(u32x4*)(dst + ((size_t)(r0 + rl) * D + pb) * esz + cb) = *(const u32x4*)(stage + rl * 32 * esz + cb);
                    }
                } else if (lane == 0) {
                    *(u32x2*)dst = *(const u32x2*)stage;   // N = 0, binary32 output
                }
            }
            __syncthreads();
            continue;
        }
        const uint32_t run = D < 32u ? D * D : 1024u;
        unsigned char* o = dst + (size_t)pauli_index(X0, pb) * esz;
        if (pb < D) {
            if (run * esz >= 16) {
                for (uint32_t b = lane * 16; b < run * esz; b += 64 * 16) *(u32x4*)(o + b) = *(const u32x4*)(stage + b);
            } else if (lane == 0) {
                *(u32x2*)o = *(const u32x2*)stage;   // N = 0, binary32 output
            }
            if (HERM && pair) {   // 1024-runs only: 2^b >= 512 rows, so N >= 10
                unsigned char* o2 = dst + (size_t)pauli_index(X0, pb ^ pair) * esz;
                for (uint32_t b = lane * 16; b < run * esz; b += 64 * 16) *(u32x4*)(o2 + b) = *(const u32x4*)(stage2 + b);
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t i8_workspace_bytes(int N, int batch) {
    return round256(i8_packed_bytes(N) * (size_t)batch) + round256(sizeof(I8Scale) * (size_t)batch) +
           sizeof(double) * i8_absmax_blocks(N) * (size_t)batch;
}

hipError_t launch_i8_pack(const void* in, bool in128, int N, int batch, void* ws, Dir dir, bool herm,
                          hipStream_t s) {
    uint32_t R = i8_absmax_blocks(N);
    double* partial = i8_partials(ws, N, batch);
    I8Scale* rec = i8_scales(ws, N, batch);
    const uint32_t half = (1u << N) / 2u;
    if (herm && half >= 1u) {
        R = R < half ? R : half;   // both powers of two: R divides D / 2
        if (in128) hipLaunchKernelGGL((i8_absmax_lower_kernel<true>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
        else hipLaunchKernelGGL((i8_absmax_lower_kernel<false>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    } else if (in128) {
        hipLaunchKernelGGL((i8_absmax_kernel<true>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    } else {
        hipLaunchKernelGGL((i8_absmax_kernel<false>), dim3(R, batch), dim3(256), 0, s, in, N, partial, R);
    }
    hipLaunchKernelGGL(i8_scale_kernel, dim3(batch), dim3(256), 0, s, (const double*)partial, R, rec);
    if (dir == ADJOINT) {
        auto kern = in128 ? i8_pack_adj_kernel<true> : i8_pack_adj_kernel<false>;
        hipLaunchKernelGGL(kern, dim3(pack_tiles(N), batch), dim3(256), 0, s, in, ws, N, (const I8Scale*)rec);
        return hipGetLastError();
    }
    const uint32_t ptiles = herm ? herm_pack_tiles(N, I8_HERM_FROM) : pack_tiles(N);
    auto kern = in128 ? (herm ? i8_pack_kernel<true, true> : i8_pack_kernel<true, false>)
                      : (herm ? i8_pack_kernel<false, true> : i8_pack_kernel<false, false>);
    hipLaunchKernelGGL(kern, dim3(ptiles, batch), dim3(256), 0, s, in, ws, N, (const I8Scale*)rec);
    return hipGetLastError();
}

template <bool HERM, bool ADJ>
hipError_t launch_i8_contract_t(const void* ws, void* out, bool out128, int N, int batch, double scale,
                                hipStream_t s) {
    constexpr int WAVES = i8_waves(HERM), MT = i8_rows(HERM);
    const uint32_t Dp = padded_dim(N);
    const uint32_t nMB = (Dp + MT - 1) / MT, nXB = Dp / XT;
    const int lds = WAVES * 1024 * (out128 ? 16 : 8) * (HERM ? 2 : 1);
    // slices per slab: a power of two, so a multiple of the step it is given
    const uint32_t nS = Dp / I8_SK;
    auto kern = nS >= (uint32_t)I8_STEP ? i8_contract_kernel<I8_STEP, HERM, ADJ>
                                        : (nS >= 8u ? i8_contract_kernel<8, HERM, ADJ> : i8_contract_kernel<1, HERM, ADJ>);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    I8Params p = {ws, out, N, out128 ? 1 : 0, scale, i8_scales(const_cast<void*>(ws), N, batch)};
    hipLaunchKernelGGL(kern, dim3(nMB * nXB, batch), dim3(WAVES * 64), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_i8_contract(const void* ws, void* out, bool out128, int N, int batch, double scale, Dir dir,
                              bool herm, hipStream_t s) {
    if (dir == ADJOINT) return launch_i8_contract_t<false, true>(ws, out, out128, N, batch, scale, s);
    return herm ? launch_i8_contract_t<true, false>(ws, out, out128, N, batch, scale, s)
                : launch_i8_contract_t<false, false>(ws, out, out128, N, batch, scale, s);
}

hipError_t launch_i8(Dir dir, const void* in, bool in128, void* out, bool out128, int N, int batch, double scale,
                     void* ws, bool herm, hipStream_t s) {
    hipError_t e = launch_i8_pack(in, in128, N, batch, ws, dir, herm, s);
    if (e != hipSuccess) return e;
    return launch_i8_contract(ws, out, out128, N, batch, scale, dir, herm, s);
}

}  // namespace pauli
