// Coefficients of a caller-given list of Pauli strings: for each n,
//   c_n = 2^-N (-i)^{popc(x&z)} sum_i (-1)^{popc(i&z)} G[i^x][i]
// with (x, z) the flip and phase masks of n -- the O(2^N) inner product of a
// matrix with one Pauli string (T. Jones 2024, sections 3 and 4), summed in
// binary64.
//
// Memory layout argument: the host groups the strings into line groups, the
// flip masks that agree above bit 3 (x >> 4).  For an aligned block of 16
// columns i0..i0+15, the rows i ^ x of the 16 masks of one line group are the
// same 16 rows, and each of the 16 entries of those rows inside the block
// lies on the diagonal of exactly one of the masks.  So the 16 x 16 tile is
// read whole (sixteen full 128-byte lines for complex64) and every byte of it
// is used: a line group costs one pass over 16 * 2^N elements of G however
// many of its strings are requested.
//
// Grid (chunk, part): a chunk is at most 256 strings of one line group (host
// plan); its columns are processed in batches of IB, and part p of P takes
// batches p, p + P, ... (in an order rotated per chunk).  A workgroup stages
// each batch's tiles in LDS, transposed to v[x & 15][i], while the next two
// batches' loads are in flight; then every string is summed by T = 256 /
// pow2ceil(count) threads over a strided share of the batch.  The T partial
// sums are reduced with lane shuffles (through LDS when T > 64) in a fixed
// order.  With P = 1 the workgroup applies the phase and 2^-N and stores the
// coefficient; with P > 1 it stores its partial sum and strings_finish adds
// the P parts in a fixed order.  Results are therefore bit-reproducible for
// a given list.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace {

constexpr int IB = 128;          // columns per LDS batch
// A full batch (16 rows x IB columns) is exactly 8 elements per thread of the
// 256-thread gather below, which loads them without bounds tests.
static_assert(IB * 16 == 8 * 256, "the unguarded gather covers exactly one batch");

// LDS row pitch (binary64 complex elements): rows start 64 bytes (16 banks)
// apart, so the row segments that the strings of one 16-lane read phase touch
// do not collide.  Columns are staged already widened to binary64, so the
// per-string sums read them without a conversion (each staged value feeds
// every string of its flip mask).
constexpr int PITCH = IB + 64 / 16;

__device__ inline double flip_sign(double a, uint32_t neg) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, a) ^ ((uint64_t)neg << 63));
}

// One batch of the gather: element e = tid + 256 j of the ib x W batch is
// (block b, tile row r, tile column c).  FULL: D >= IB, so all 8 elements
// exist and no test is needed (this keeps the loads unconditional, so the
// compiler can count them and wait only for the batch being staged).
template <typename InT, bool FULL>
__device__ __attribute__((always_inline)) inline void fetch_batch(const InT* __restrict__ G, uint32_t D, uint32_t W,
                                                                  uint32_t lw, uint32_t ib, uint32_t x0, uint32_t i0,
                                                                  int tid, InT (&f)[8]) {
    const uint32_t total = ib * W;
#pragma clang loop unroll(full)
    for (int j = 0; j < 8; ++j) {
        const uint32_t e = (uint32_t)tid + 256u * j;
        if (FULL || e < total) {
            const uint32_t c = e & (W - 1u), r = (e >> lw) & (W - 1u), b = e >> (2 * lw);
            const uint32_t col = i0 + (b << lw) + c;
            const uint32_t row = ((i0 + (b << lw)) ^ x0) + r;
            const InT g = G[(size_t)row * D + col];
            f[j].x = g.x;
            f[j].y = g.y;
        }
    }
}

// Write a fetched batch to LDS transposed to v[x & 15][column], in binary64.
template <typename InT, bool FULL>
__device__ __attribute__((always_inline)) inline void stage_batch(double2* v, uint32_t W, uint32_t lw, uint32_t ib,
                                                                  int tid, const InT (&f)[8]) {
    const uint32_t total = ib * W;
#pragma clang loop unroll(full)
    for (int j = 0; j < 8; ++j) {
        const uint32_t e = (uint32_t)tid + 256u * j;
        if (FULL || e < total) {
            const uint32_t c = e & (W - 1u), r = (e >> lw) & (W - 1u), b = e >> (2 * lw);
            double2& d = v[(r ^ c) * PITCH + (b << lw) + c];
            d.x = (double)f[j].x;
            d.y = (double)f[j].y;
        }
    }
}

template <typename InT>
__global__ __launch_bounds__(256) void strings_kernel(const InT* __restrict__ G, int N,
                                                      const StringChunk* __restrict__ chunks,
                                                      const StringEntry* __restrict__ entries,
                                                      void* __restrict__ out, int out128, double scale,
                                                      double2* __restrict__ partial, uint32_t count_total) {
    __shared__ double2 v[16 * PITCH];
    __shared__ double part[4][2];

    const uint32_t D = 1u << N;
    const uint32_t W = D < 16u ? D : 16u;          // line-group width (masks and columns)
    const uint32_t lw = D < 16u ? (uint32_t)N : 4u;
    const uint32_t ib = D < (uint32_t)IB ? D : (uint32_t)IB;
    const uint32_t nb = D / ib;                    // column batches
    const uint32_t P = gridDim.y, p = blockIdx.y;
    const StringChunk ch = chunks[blockIdx.x];
    const int tid = threadIdx.x;

    int sp = 1;
    while (sp < (int)ch.count) sp <<= 1;           // count is in 1..256
    const int T = 256 / sp;                        // threads per string (power of two)
    const int s = tid / T, q = tid % T;
    const bool has = s < (int)ch.count;
    uint32_t n = 0;
    if (has) n = entries[ch.first + s].n;
    const uint32_t x = flip_of_index(n), z = phase_of_index(n);
    const double2* vrow = v + (x & (W - 1u)) * PITCH;

    double re = 0.0, im = 0.0;
    // Columns il = q + T (8u + t) of a batch, t < 8.  The bits of q, T t,
    // 8 T u and the batch offset b ib are disjoint, so the sign
    // (-1)^{popc(i & z)} is a per-thread factor st[t], fixed for the whole
    // pass, times one factor per group of 8 columns; every product with +-1
    // is exact, and each column costs two fused multiply-adds.
    int lt = 0;
    while ((1 << lt) < T) ++lt;
    double st[8];
    {
        const uint32_t zq = (uint32_t)__popc((uint32_t)q & z);
#pragma unroll
        for (int t = 0; t < 8; ++t)
            st[t] = ((zq + (uint32_t)__popc(((uint32_t)t << lt) & z)) & 1u) ? -1.0 : 1.0;
    }
    auto batch_sum = [&](uint32_t b) {
        if (!has) return;
        const uint32_t par0 = (uint32_t)__popc((b * ib) & z);
        if (ib >= 8u * (uint32_t)T) {           // uniform: T and ib are per-workgroup
            const uint32_t step = 8u * (uint32_t)T;
            for (uint32_t g0 = 0; g0 < ib; g0 += step) {
                const double2* src = vrow + g0 + (uint32_t)q;
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const double2 g = src[t << lt];
                    sr = fma(g.x, st[t], sr);
                    si = fma(g.y, st[t], si);
                }
                const double su = ((par0 + (uint32_t)__popc(g0 & z)) & 1u) ? -1.0 : 1.0;
                re = fma(sr, su, re);
                im = fma(si, su, im);
            }
        } else {                                // fewer than 8 columns per thread
            for (uint32_t il = q; il < ib; il += T) {
                const double2 g = vrow[il];
                const uint32_t neg = (par0 + (uint32_t)__popc(il & z)) & 1u;
                re += flip_sign(g.x, neg);
                im += flip_sign(g.y, neg);
            }
        }
    };
    // Part p takes batches p, p + P, ... (m of them), visited from a start
    // rotated by the chunk index so that concurrent chunks read different
    // column ranges of G.  Two batches in flight: while one is summed, the
    // next two load.
    const uint32_t m = p < nb ? (nb - 1u - p) / P + 1u : 0u;
    const uint32_t rot = m ? blockIdx.x % m : 0u;
    auto batch_at = [&](uint32_t k) { return p + P * ((k + rot) % m); };
    auto run = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        InT f0[8], f1[8];   // one batch of the gather each, 8 elements per thread
        if (m > 0) fetch_batch<InT, FULL>(G, D, W, lw, ib, ch.x0, batch_at(0) * ib, tid, f0);
        if (m > 1) fetch_batch<InT, FULL>(G, D, W, lw, ib, ch.x0, batch_at(1) * ib, tid, f1);
        for (uint32_t k = 0; k < m; k += 2) {
            stage_batch<InT, FULL>(v, W, lw, ib, tid, f0);
            __syncthreads();
            if (k + 2 < m) fetch_batch<InT, FULL>(G, D, W, lw, ib, ch.x0, batch_at(k + 2) * ib, tid, f0);
            batch_sum(batch_at(k));
            __syncthreads();   // the next stage_batch overwrites v
            if (k + 1 >= m) break;
            stage_batch<InT, FULL>(v, W, lw, ib, tid, f1);
            __syncthreads();
            if (k + 3 < m) fetch_batch<InT, FULL>(G, D, W, lw, ib, ch.x0, batch_at(k + 3) * ib, tid, f1);
            batch_sum(batch_at(k + 1));
            __syncthreads();
        }
    };
    if (D >= (uint32_t)IB) run(std::true_type{});
    else run(std::false_type{});

    // sum over the T threads of each string (aligned groups of consecutive lanes)
    for (int off = 1; off < T && off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if (T > 64) {          // uniform: one or two strings spread over several waves
        if ((tid & 63) == 0) {
            part[tid >> 6][0] = re;
            part[tid >> 6][1] = im;
        }
        __syncthreads();
        if (q == 0) {
            re = 0.0;
            im = 0.0;
            for (int w = 0; w < T / 64; ++w) {
                re += part[(tid >> 6) + w][0];
                im += part[(tid >> 6) + w][1];
            }
        }
    }
    if (!has || q != 0) return;
    if (P > 1) {
        partial[(size_t)p * count_total + ch.first + s] = make_double2(re, im);
        return;
    }
    rotate_minus_i(re, im, (uint32_t)__popc(x & z));
    re *= scale;
    im *= scale;
    const uint32_t slot = entries[ch.first + s].slot;
    if (out128) ((double2*)out)[slot] = make_double2(re, im);
    else ((float2*)out)[slot] = make_float2((float)re, (float)im);
}

// P > 1: add the P parts of every entry, then phase and 2^-N.  Few parts:
// one thread per entry, parts in order.  Many parts (FINISH_WAVE_PARTS or
// more): one wavefront per entry, lane l adding parts l, l + 64, ... in order
// before a fixed butterfly over the lanes.
constexpr uint32_t FINISH_WAVE_PARTS = 16;

__device__ inline void finish_store(const StringEntry& e, double re, double im, void* out, int out128,
                                    double scale) {
    rotate_minus_i(re, im, (uint32_t)__popc(flip_of_index(e.n) & phase_of_index(e.n)));
    re *= scale;
    im *= scale;
    if (out128) ((double2*)out)[e.slot] = make_double2(re, im);
    else ((float2*)out)[e.slot] = make_float2((float)re, (float)im);
}

__global__ __launch_bounds__(256) void strings_finish(const StringEntry* __restrict__ entries,
                                                      const double2* __restrict__ partial, uint32_t count,
                                                      uint32_t P, void* __restrict__ out, int out128,
                                                      double scale) {
    double re = 0.0, im = 0.0;
    if (P < FINISH_WAVE_PARTS) {
        const uint32_t k = blockIdx.x * 256u + threadIdx.x;
        if (k >= count) return;
        for (uint32_t p = 0; p < P; ++p) {
            const double2 a = partial[(size_t)p * count + k];
            re += a.x;
            im += a.y;
        }
        finish_store(entries[k], re, im, out, out128, scale);
        return;
    }
    const uint32_t k = blockIdx.x * 4u + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
    if (k >= count) return;                        // uniform per wavefront
    for (uint32_t p = lane; p < P; p += 64u) {
        const double2 a = partial[(size_t)p * count + k];
        re += a.x;
        im += a.y;
    }
    for (int off = 1; off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if (lane == 0) finish_store(entries[k], re, im, out, out128, scale);
}

}  // namespace

uint32_t strings_batches(int N) {
    const uint32_t D = 1u << N;
    return D < (uint32_t)IB ? 1u : D / IB;
}

hipError_t launch_strings(const void* G, bool in_c128, int N, const StringChunk* chunks, int nchunks,
                          const StringEntry* entries, int count, int parts, double2* partial, void* out,
                          bool out_c128, hipStream_t stream) {
    const double scale = 1.0 / (double)(1u << N);
    const dim3 grid((uint32_t)nchunks, (uint32_t)parts);
    if (in_c128)
        hipLaunchKernelGGL(strings_kernel<double2>, grid, dim3(256), 0, stream, (const double2*)G, N, chunks,
                           entries, out, out_c128 ? 1 : 0, scale, partial, (uint32_t)count);
    else
        hipLaunchKernelGGL(strings_kernel<float2>, grid, dim3(256), 0, stream, (const float2*)G, N, chunks,
                           entries, out, out_c128 ? 1 : 0, scale, partial, (uint32_t)count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || parts == 1) return e;
    const uint32_t per_block = (uint32_t)parts < FINISH_WAVE_PARTS ? 256u : 4u;
    hipLaunchKernelGGL(strings_finish, dim3(((uint32_t)count + per_block - 1u) / per_block), dim3(256), 0, stream, entries,
                       (const double2*)partial, (uint32_t)count, (uint32_t)parts, out, out_c128 ? 1 : 0, scale);
    return hipGetLastError();
}

}  // namespace pauli

// ---- adjoint of the list: grad_G = 2^-N sum_k g_k P_{n_k} ----
namespace pauli {
namespace {

// One workgroup per (line group of 16 flip masks, batch of 128 columns):
// every entry G[i ^ x][i] of the 16 x 128 block gets
//   2^-N sum over listed strings k with flip mask x of
//        i^{popc(x&z_k)} (-1)^{popc(i&z_k)} g_k,
// zero when no listed string has flip mask x.  Element e = t + 256 j is
// (column block c_b = e >> 8, row r, column c of its 16 x 16 tile), x_l =
// r ^ c; sixteen consecutive threads write one 128-byte row segment.
// first[x] .. first[x + 1] are the positions of mask x's strings in entries.
template <bool GRAD128, bool OUT128>
__global__ __launch_bounds__(256) void strings_adjoint(const void* __restrict__ grad, const StringEntry* __restrict__ entries,
                                                       const uint32_t* __restrict__ first, void* __restrict__ out,
                                                       int N, double scale) {
    const uint32_t D = 1u << N;
    const uint32_t W = D < 16u ? D : 16u, lw = D < 16u ? (uint32_t)N : 4u;
    const uint32_t ib = D < 128u ? D : 128u;
    const uint32_t x0 = blockIdx.y * W, i0 = blockIdx.x * ib;
    const uint32_t total = ib * W;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t e = threadIdx.x + 256u * j;
        if (e >= total) break;
        const uint32_t c = e & (W - 1u), r = (e >> lw) & (W - 1u), b = e >> (2 * lw);
        const uint32_t col = i0 + (b << lw) + c;
        const uint32_t x = x0 + (r ^ c);
        const uint32_t row = col ^ x;
        double re = 0.0, im = 0.0;
        for (uint32_t k = first[x]; k < first[x + 1]; ++k) {
            const StringEntry s = entries[k];
            const uint32_t z = phase_of_index(s.n);
            double gr, gi;
            if constexpr (GRAD128) {
                const double2 g = ((const double2*)grad)[s.slot];
                gr = g.x;
                gi = g.y;
            } else {
                const float2 g = ((const float2*)grad)[s.slot];
                gr = (double)g.x;
                gi = (double)g.y;
            }
            rotate_minus_i(gr, gi, 3u * (uint32_t)__popc(x & z) + 2u * (uint32_t)__popc(col & z));
            re += gr;
            im += gi;
        }
        re *= scale;
        im *= scale;
        if constexpr (OUT128) ((double2*)out)[(size_t)row * D + col] = make_double2(re, im);
        else ((float2*)out)[(size_t)row * D + col] = make_float2((float)re, (float)im);
    }
}

}  // namespace

hipError_t launch_strings_adjoint(const void* grad, bool grad_c128, const StringEntry* entries,
                                  const uint32_t* first, void* out, bool out_c128, int N, hipStream_t stream) {
    const uint32_t D = 1u << N;
    const uint32_t W = D < 16u ? D : 16u, ib = D < 128u ? D : 128u;
    const dim3 grid(D / ib, D / W);
    const double scale = 1.0 / (double)D;
    if (grad_c128) {
        if (out_c128)
            hipLaunchKernelGGL((strings_adjoint<true, true>), grid, dim3(256), 0, stream, grad, entries, first, out, N, scale);
        else
            hipLaunchKernelGGL((strings_adjoint<true, false>), grid, dim3(256), 0, stream, grad, entries, first, out, N, scale);
    } else {
        if (out_c128)
            hipLaunchKernelGGL((strings_adjoint<false, true>), grid, dim3(256), 0, stream, grad, entries, first, out, N, scale);
        else
            hipLaunchKernelGGL((strings_adjoint<false, false>), grid, dim3(256), 0, stream, grad, entries, first, out, N, scale);
    }
    return hipGetLastError();
}

}  // namespace pauli
