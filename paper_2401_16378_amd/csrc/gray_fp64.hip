// Binary64 VALU kernel: every coefficient summed sequentially in Gray-code
// order with the one-sign recurrence, as the paper's algorithm does
// (section 3, Fig. 1b; Eq. (c_def_in_terms_of_fn) and
// Eq. (lambda_recurrence_over_i)).
//
// Mapping.  A wave's 64 lanes own 64 consecutive flip masks x; the wave owns
// 16 consecutive "row" indices p (phase masks z in the forward direction,
// matrix columns i in the adjoint).  For the summation index q (i forward,
// z adjoint) visited as q = gray(k), the sign (-1)^{popc(q & p)} of lane-row
// p = P + j factorises into a part fixed by the low 4 bits (j, known when the
// walk is unrolled) and a part sigma shared by the wave (high bits of P) that
// the recurrence flips only at steps whose changed bit t >= 4.  Every term is
// therefore one FMA of an exact +-1 with the input value, the same rounding
// as the paper's  c += lambda * G  in the same order: the result matches the
// sequential Gray-order sum bit for bit.  The constant phase (-i)^{popc(x&z)}
// and the 2^-N factor are exact and applied at the end (forward) or on load
// (adjoint, i^{popc(x&z)}).
//
// Data path.  The input for a chunk of IC = 32 consecutive walk steps (an
// aligned block of q, since Gray codes map aligned blocks of k onto aligned
// blocks of q) and the block's 64 x's is staged in LDS as binary64 pairs,
// rows in walk order, double-buffered.  The forward chunk is an aligned
// 64 x 32 region of G read along rows; the adjoint chunk is a run of
// contiguous coefficient blocks.  Each step is one LDS read per lane and
// 32 FMAs per lane, so the kernel is bound by binary64 VALU throughput.
#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace {

constexpr int ROWS_PER_WAVE = 16;

__device__ inline double2 load_c(const float2* p) {
    float2 v = *p;
    return make_double2((double)v.x, (double)v.y);
}
__device__ inline double2 load_c(const double2* p) { return *p; }
__device__ inline void store_c(float2* p, double re, double im) {
    *p = make_float2((float)re, (float)im);
}
__device__ inline void store_c(double2* p, double re, double im) { *p = make_double2(re, im); }

template <int LOG_IC, int WAVES, int DIR, typename InT, typename OutT>
__global__ __launch_bounds__(WAVES * 64) void gray_kernel(const InT* __restrict__ in,
                                                          OutT* __restrict__ out, int N,
                                                          double scale) {
    constexpr int IC = 1 << LOG_IC;
    constexpr int NT = WAVES * 64;
    constexpr int PPG = WAVES * ROWS_PER_WAVE;            // rows p per workgroup
    constexpr int EPT = (IC * 64 + NT - 1) / NT;          // staged elements per thread
    extern __shared__ double2 lds[];                      // [2][IC][64]

    const uint32_t D = 1u << N;
    const uint32_t XB = D < 64u ? D : 64u;
    const uint32_t nPG = (D + PPG - 1) / PPG;
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t xb = L / nPG, pg = L % nPG;
    const uint32_t X0 = xb * XB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t P = pg * PPG + wave * ROWS_PER_WAVE;  // first row of this wave

    const size_t mat = (size_t)D * D;
    const InT* src = in + (size_t)blockIdx.y * mat;
    OutT* dst = out + (size_t)blockIdx.y * mat;
    const uint32_t nchunks = D >> LOG_IC;
    const uint32_t chunk_elems = (uint32_t)IC * XB;

    double2 stage[EPT];
    uint32_t spos[EPT];

    // Fetch chunk kb into registers; record where each element lands in LDS.
    auto fetch = [&](uint32_t kb) {
        const uint32_t Q0 = gray(kb) << LOG_IC;
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const uint32_t e = (uint32_t)tid + (uint32_t)s * NT;
            spos[s] = 0xFFFFFFFFu;
            if (e < chunk_elems) {
                uint32_t q, xl;
                double2 v;
                if (DIR == FORWARD) {
                    // aligned XB x IC region of G: rows (Q0^X0) & ~(XB-1) .., columns Q0 ..
                    const uint32_t R0 = (Q0 ^ X0) & ~(XB - 1u);
                    const uint32_t r = R0 + e / IC, c = e % IC;
                    q = Q0 + c;
                    xl = (r ^ q) - X0;
                    v = load_c(src + (size_t)r * D + q);
                } else {
                    // XB/IC contiguous runs of IC*IC coefficients
                    const uint32_t sq = e / (IC * IC), o = e % (IC * IC);
                    const uint32_t zl = compact_even(o >> 1);
                    const uint32_t x = X0 + sq * IC + (compact_even(o) ^ zl);
                    q = Q0 + zl;
                    xl = x - X0;
                    v = load_c(src + pauli_index(x, q));
                    // i^{popc(x&z)} = (-i)^{3 popc(x&z)}
                    rotate_minus_i(v.x, v.y, 3u * (uint32_t)__popc(x & q));
                }
                stage[s] = v;
                spos[s] = (gray_inverse(q) & (IC - 1)) * 64 + xl;
            }
        }
    };
    auto deposit = [&](int buf) {
#pragma unroll
        for (int s = 0; s < EPT; ++s)
            if (spos[s] != 0xFFFFFFFFu) lds[buf * IC * 64 + spos[s]] = stage[s];
    };

    double acc_re[ROWS_PER_WAVE], acc_im[ROWS_PER_WAVE];
#pragma unroll
    for (int j = 0; j < ROWS_PER_WAVE; ++j) acc_re[j] = acc_im[j] = 0.0;
    double sigma = 1.0;

    fetch(0);
    deposit(0);
    __syncthreads();
    for (uint32_t kb = 0; kb < nchunks; ++kb) {
        const int buf = kb & 1;
        if (kb + 1 < nchunks) fetch(kb + 1);
        if (kb > 0) {
            // step k = kb*IC changes bit t = ctz(k) >= LOG_IC (>= 5 here)
            const int t = __builtin_ctz(kb) + LOG_IC;
            if ((P >> t) & 1u) sigma = -sigma;
        }
        const double2* row = lds + buf * IC * 64 + lane;
#pragma unroll
        for (int kl = 0; kl < IC; ++kl) {
            if (kl == 16) {
                // step changing bit 4: flips the rows whose bit 4 is set (all or none)
                if ((P >> 4) & 1u) sigma = -sigma;
            }
            const double2 v = row[kl * 64];
            const uint32_t g = gray((uint32_t)kl) & 15u;
#pragma unroll
            for (int j = 0; j < ROWS_PER_WAVE; ++j) {
                const double s = (popc_const(g & (uint32_t)j) & 1) ? -sigma : sigma;
                acc_re[j] = __builtin_fma(s, v.x, acc_re[j]);
                acc_im[j] = __builtin_fma(s, v.y, acc_im[j]);
            }
        }
        if (kb + 1 < nchunks) deposit(buf ^ 1);
        __syncthreads();
    }

    if ((uint32_t)lane >= XB) return;
    const uint32_t x = X0 + lane;
#pragma unroll
    for (int j = 0; j < ROWS_PER_WAVE; ++j) {
        const uint32_t p = P + j;
        if (p >= D) continue;
        double re = acc_re[j], im = acc_im[j];
        if (DIR == FORWARD) {
            rotate_minus_i(re, im, (uint32_t)__popc(x & p));
            store_c(dst + pauli_index(x, p), re * scale, im * scale);
        } else {
            store_c(dst + (size_t)(p ^ x) * D + p, re * scale, im * scale);
        }
    }
}

template <int LOG_IC, int WAVES, int DIR, typename InT, typename OutT>
hipError_t launch_t(const void* in, void* out, int N, int batch, double scale, hipStream_t s) {
    constexpr int PPG = WAVES * ROWS_PER_WAVE;
    const uint32_t D = 1u << N;
    const uint32_t XB = D < 64u ? D : 64u;
    const uint32_t nPG = (D + PPG - 1) / PPG;
    const uint32_t blocks = (D / XB) * nPG;
    const size_t lds_bytes = 2 * (size_t)(1 << LOG_IC) * 64 * sizeof(double2);
    auto kern = gray_kernel<LOG_IC, WAVES, DIR, InT, OutT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks, batch), dim3(WAVES * 64), lds_bytes, s,
                       (const InT*)in, (OutT*)out, N, scale);
    return hipGetLastError();
}

template <int DIR, typename InT, typename OutT>
hipError_t launch_dir(const void* in, void* out, int N, int batch, double scale, hipStream_t s) {
    // The walk is unrolled per chunk of 2^min(N,5) steps; more than one chunk
    // only occurs with the full 32-step chunk.
    if (N >= 12) return launch_t<5, 8, DIR, InT, OutT>(in, out, N, batch, scale, s);
    if (N >= 6) return launch_t<5, 4, DIR, InT, OutT>(in, out, N, batch, scale, s);
    switch (N) {
        case 5: return launch_t<5, 2, DIR, InT, OutT>(in, out, N, batch, scale, s);
        case 4: return launch_t<4, 1, DIR, InT, OutT>(in, out, N, batch, scale, s);
        case 3: return launch_t<3, 1, DIR, InT, OutT>(in, out, N, batch, scale, s);
        case 2: return launch_t<2, 1, DIR, InT, OutT>(in, out, N, batch, scale, s);
        case 1: return launch_t<1, 1, DIR, InT, OutT>(in, out, N, batch, scale, s);
        default: return launch_t<0, 1, DIR, InT, OutT>(in, out, N, batch, scale, s);
    }
}

template <int DIR>
hipError_t launch_types(const void* in, bool in128, void* out, bool out128, int N, int batch,
                        double scale, hipStream_t s) {
    if (in128 && out128) return launch_dir<DIR, double2, double2>(in, out, N, batch, scale, s);
    if (in128) return launch_dir<DIR, double2, float2>(in, out, N, batch, scale, s);
    if (out128) return launch_dir<DIR, float2, double2>(in, out, N, batch, scale, s);
    return launch_dir<DIR, float2, float2>(in, out, N, batch, scale, s);
}

}  // namespace

hipError_t launch_gray(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N,
                       int batch, double scale, hipStream_t stream) {
    if (dir == FORWARD)
        return launch_types<FORWARD>(in, in_c128, out, out_c128, N, batch, scale, stream);
    return launch_types<ADJOINT>(in, in_c128, out, out_c128, N, batch, scale, stream);
}

}  // namespace pauli
