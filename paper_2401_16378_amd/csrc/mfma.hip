// Matrix-core (MFMA) path for gfx950: the paper's O(2^N)-per-coefficient
// sum (Eq. (c_def_in_terms_of_fn)) for all coefficients at once, i.e. the
// O(8^N) total of section 3, evaluated as a dense contraction
//
//     C[p][x] = sum_q H[p][q] * In[q][x],      H[p][q] = (-1)^{popc(p & q)}
//
// forward (decomposition):  q = i, p = z, In[i][x] = G[i^x][i] (the gathered
//   XOR diagonal v_x), out[n(x,z)] = 2^-N (-i)^{popc(x&z)} C[z][x];
// adjoint (recomposition / gradient):  q = z, p = i,
//   In[z][x] = i^{popc(x&z)} c[n(x,z)],  G[i^x][i] = scale * C[i][x].
//
// H is the Sylvester-Hadamard sign matrix: every entry is +-1, exact in any
// format, so it never touches memory.  Over an aligned 32-row block it is
// one fixed 32x32 block times a sign fixed by the blocks' high bits; the
// kernel keeps the two fragments of that block (and their negations) in
// registers and picks them at compile time, with one extra sign per wave and
// K-tile.
//
// Precision.  PLANES = 3: each binary32 component g is split as
// g ~ hi + mid + lo (three bf16 numbers, hi on a power-of-two grid shared by
// the 4x4 micro-block, see split3); bf16 MFMA accumulates hi into one FP32
// accumulator, where the sums stay exact, and mid + lo into a second, and the
// two are added in binary64 in the epilogue before the phase and scale.  PLANES = 1: binary32 MFMA on
// the binary32 components.
//
// Tiling.  A workgroup owns 32 flip masks x (64 real B columns: re then im)
// and WAVES*RB*32 rows p; each wave owns RB*32 rows and the whole K range.
// K is walked in tiles of KT = 32*RB, staged through double-buffered LDS.
// A thread loads one aligned 4x4 micro-block per K-tile: in the forward
// direction 4 rows x 4 columns of G, which the XOR map sends to 4 columns x
// 4 consecutive q of In; in the adjoint, 16 consecutive coefficients, which
// form a 4x4 (z,x) block.  Each LDS write is therefore 4 consecutive q of one
// column: 8 bytes per bf16 plane, 16 bytes for fp32.
#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int XT = 32;  // flip masks per workgroup

__device__ inline uint32_t pack_bf16(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline float lo_half(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_half(uint32_t u) { return __builtin_bit_cast(float, u & 0xFFFF0000u); }

// Three-way bf16 split of two binary32 values a, b against a power-of-two
// grid u (with inv_u = 1/u, both exact):
//   hi  = u * rint(x / u)        (|x| < 256 u, so hi has <= 8 significant bits
//                                 and is exact in bf16)
//   mid = bf16(x - hi),  lo = bf16(x - hi - mid)
// x - hi and x - hi - mid are exact in binary32, so hi + mid + lo carries
// every bit of x except at most those below 2^-17 |x - hi|.  All hi terms of
// a micro-block are multiples of the same u, which keeps the FP32 sums of hi
// terms exact over the whole K range for any input whose partial sums stay
// below 2^24 times the smallest grid (about 2^16 times the smallest block
// maximum), instead of rounding away the low bits of small terms.
__device__ inline void split3(float a, float b, float u, float inv_u, uint32_t& h, uint32_t& m,
                              uint32_t& l) {
    const float ha = __builtin_rintf(a * inv_u) * u, hb = __builtin_rintf(b * inv_u) * u;
    h = pack_bf16(ha, hb);
    const float ra = a - ha, rb = b - hb;
    m = pack_bf16(ra, rb);
    const float qa = ra - lo_half(m), qb = rb - hi_half(m);
    l = pack_bf16(qa, qb);
}

// Grid of a micro-block: u = 2^(e-8) for the exponent e with max|x| < 2^e,
// clamped so that u and 1/u stay normal binary32 numbers.
__device__ inline void block_grid(float maxabs, float& u, float& inv_u) {
    int e = (int)((__builtin_bit_cast(uint32_t, maxabs) >> 23) & 0xFFu) - 126;
    e = e < -110 ? -110 : (e > 120 ? 120 : e);
    u = __builtin_bit_cast(float, (uint32_t)(127 + e - 8) << 23);
    inv_u = __builtin_bit_cast(float, (uint32_t)(127 - e + 8) << 23);
}

template <int PLANES, int RB, int WAVES>
struct Cfg {
    static constexpr int KT = 32 * RB;                 // K per tile
    static constexpr int NT = WAVES * 64;              // threads
    static constexpr int MT = WAVES * RB * 32;         // rows per workgroup
    static constexpr int NPL = PLANES == 3 ? 6 : 2;    // LDS planes (plane x re/im)
    static constexpr int ESZ = PLANES == 3 ? 2 : 4;    // bytes per LDS element
    static constexpr int PITCH = KT * ESZ + 16;        // bytes per LDS column (padded)
    static constexpr int BUF = NPL * XT * PITCH;       // bytes per K-tile buffer
    static constexpr int UBLK = 2 * KT;                // 4x4 micro-blocks per K-tile
    static constexpr int UPT = (UBLK + NT - 1) / NT;   // micro-blocks per thread
    static int lds_bytes(int esz) {                     // K-tile buffers or epilogue staging
        const int stage = WAVES * 1024 * esz;
        return 2 * BUF > stage ? 2 * BUF : stage;
    }
};

struct Params {
    const void* in;
    void* out;
    int N;
    int out128;
    double scale;
};

template <bool IN128>
__device__ inline f32x2 load_elem(const unsigned char* base, size_t idx) {
    if constexpr (IN128) {
        const double2 v = ((const double2*)base)[idx];
        return f32x2{(float)v.x, (float)v.y};
    } else {
        const float2 v = ((const float2*)base)[idx];
        return f32x2{v.x, v.y};
    }
}

template <int PLANES, int RB, int WAVES, int DIR, bool IN128>
__global__ __launch_bounds__(WAVES * 64) void mfma_kernel(Params prm) {
    using C = Cfg<PLANES, RB, WAVES>;
    constexpr int KT = C::KT;
    constexpr int ACC = PLANES == 3 ? 2 : 1;
    constexpr int UPT = C::UPT;
    constexpr int NPARTS = 4 * UPT;                          // deposit pieces per K-tile
    constexpr int S = PLANES == 3 ? KT / 16 : KT / 8;        // K-slices per tile
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

    const int N = prm.N;
    const uint32_t D = 1u << N;
    const bool full = D >= 32u;                               // no padding needed
    const uint32_t nMB = D > (uint32_t)C::MT ? D / C::MT : 1u;   // row blocks
    const uint32_t nK = D > (uint32_t)KT ? D / KT : 1u;          // K tiles
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t xb = L / nMB, mb = L % nMB;
    const uint32_t X0 = xb * XT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const uint32_t Pw = mb * C::MT + wave * RB * 32;            // first row of this wave
    const size_t mat = (size_t)D * D;
    const unsigned char* src = (const unsigned char*)prm.in + (size_t)blockIdx.y * mat * (IN128 ? 16 : 8);
    unsigned char* dst = (unsigned char*)prm.out + (size_t)blockIdx.y * mat * (prm.out128 ? 16 : 8);

    // ---- prologue pieces: fetch a K-tile into registers, deposit it into LDS ----
    f32x2 stg[UPT][16];
    float gu[UPT], ginv[UPT];
    auto fetch = [&](uint32_t kt) {
        const uint32_t Q0 = kt * KT;
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int ub = tid + u * C::NT;
            if constexpr (C::UBLK < UPT * C::NT) {
                if (ub >= C::UBLK) break;
            }
            const int g = ub >> 6, w6 = ub & 63;   // 32x32 square g of the tile, block w6 in it
            if constexpr (DIR == FORWARD) {
                const int mr = w6 >> 3, mc = w6 & 7;
                const uint32_t q0 = Q0 + 32 * g + 4 * mc;
                const uint32_t r0 = (((Q0 + 32 * g) ^ X0) & ~31u) + 4 * mr;
                if (full) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            stg[u][a * 4 + b] = load_elem<IN128>(src, (size_t)(r0 + a) * D + q0 + b);
                } else {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const uint32_t r = r0 + a, q = q0 + b;
                            stg[u][a * 4 + b] = (r < D && q < D) ? load_elem<IN128>(src, (size_t)r * D + q)
                                                                 : f32x2{0.f, 0.f};
                        }
                }
            } else {
                const uint32_t zb = Q0 + 32 * g;
                const uint32_t nb = pauli_index(X0, zb);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const uint32_t o = 16 * w6 + r;
                    const uint32_t zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
                    const uint32_t z = zb + zl, x = X0 + xl;
                    f32x2 c = {0.f, 0.f};
                    if (full || (z < D && x < D)) c = load_elem<IN128>(src, nb + o);
                    float re = c.x, im = c.y;
                    rotate_minus_i(re, im, 3u * (uint32_t)__popc(x & z));  // i^{popc(x&z)}
                    stg[u][r] = f32x2{re, im};
                }
            }
        }
    };
    // grid of micro-block u (split-bf16 only)
    auto grid = [&](int u) {
        float mx = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            mx = __builtin_fmaxf(mx, __builtin_fmaxf(__builtin_fabsf(stg[u][r].x), __builtin_fabsf(stg[u][r].y)));
        block_grid(mx, gu[u], ginv[u]);
    };
    // row x2 of micro-block u: 4 consecutive K slots of one column, all planes
    auto deposit_part = [&](int buf, int u, int x2) {
        const int ub = tid + u * C::NT;
        if constexpr (C::UBLK < UPT * C::NT) {
            if (ub >= C::UBLK) return;
        }
        const int g = ub >> 6, w6 = ub & 63;
        if constexpr (PLANES == 3) {
            if (x2 == 0) grid(u);
        }
        int xh, kh;  // column group (x_l / 4) and first K slot of the micro-block
        if constexpr (DIR == FORWARD) {
            const int mr = w6 >> 3, mc = w6 & 7;
            xh = mr ^ mc;
            kh = 32 * g + 4 * mc;
        } else {
            // 16 consecutive coefficients o = 16*w6 + r, r = (x^z)_0 | z_0<<1 | (x^z)_1<<2 | z_1<<3
            const uint32_t o = 16 * w6;
            const int zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
            xh = xl >> 2;
            kh = 32 * g + zl;
        }
        f32x2 e[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if constexpr (DIR == FORWARD) {
                e[b] = stg[u][((x2 ^ b) << 2) | b];  // row a = x2 ^ b, column b
            } else {
                const int d = x2 ^ b;                 // (x ^ z) low bits
                e[b] = stg[u][(d & 1) | ((b & 1) << 1) | ((d >> 1) << 2) | ((b >> 1) << 3)];
            }
        }
        unsigned char* cbase = lds + buf * C::BUF + (xh * 4 + x2) * C::PITCH + kh * C::ESZ;
        constexpr int PS = XT * C::PITCH;  // plane stride
        if constexpr (PLANES == 3) {
            uint32_t hr0, mr0, lr0, hr1, mr1, lr1, hi0, mi0, li0, hi1, mi1, li1;
            split3(e[0].x, e[1].x, gu[u], ginv[u], hr0, mr0, lr0);
            split3(e[2].x, e[3].x, gu[u], ginv[u], hr1, mr1, lr1);
            split3(e[0].y, e[1].y, gu[u], ginv[u], hi0, mi0, li0);
            split3(e[2].y, e[3].y, gu[u], ginv[u], hi1, mi1, li1);
            *(u32x2*)(cbase + 0 * PS) = u32x2{hr0, hr1};
            *(u32x2*)(cbase + 1 * PS) = u32x2{hi0, hi1};
            *(u32x2*)(cbase + 2 * PS) = u32x2{mr0, mr1};
            *(u32x2*)(cbase + 3 * PS) = u32x2{mi0, mi1};
            *(u32x2*)(cbase + 4 * PS) = u32x2{lr0, lr1};
            *(u32x2*)(cbase + 5 * PS) = u32x2{li0, li1};
        } else {
            *(f32x4*)(cbase) = f32x4{e[0].x, e[1].x, e[2].x, e[3].x};
            *(f32x4*)(cbase + PS) = f32x4{e[0].y, e[1].y, e[2].y, e[3].y};
        }
    };
    auto deposit_all = [&](int buf) {
#pragma unroll
        for (int u = 0; u < UPT; ++u)
#pragma unroll
            for (int x2 = 0; x2 < 4; ++x2) deposit_part(buf, u, x2);
    };

    // ---- sign fragments of the 32x32 Sylvester block ----
    // bf16: lane (row p_l = l32, half h) holds K slots q_l = 16e + 8h + j, j < 8,
    //       for the two 16-wide slices e of a 32-wide block.
    // fp32: lane holds q_l = 8e + 4h + st for slice e < 4, step st < 4.
    uint32_t fA[2][4];   // bf16 pairs, [e][j/2]
    float fF[4][4];      // fp32, [e][st]
    if constexpr (PLANES == 3) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t q0 = 16 * e + 8 * h + 2 * jj;
                const uint32_t s0 = (__popc(l32 & q0) & 1) ? 0xBF80u : 0x3F80u;
                const uint32_t s1 = (__popc(l32 & (q0 + 1)) & 1) ? 0xBF80u : 0x3F80u;
                fA[e][jj] = s0 | (s1 << 16);
            }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int st = 0; st < 4; ++st)
                fF[e][st] = (__popc(l32 & (8 * e + 4 * h + st)) & 1) ? -1.f : 1.f;
    }

    f32x16 acc[ACC][RB][2];
#pragma unroll
    for (int a = 0; a < ACC; ++a)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][rb][cb][r] = 0.f;

    fetch(0);
    deposit_all(0);
    __syncthreads();
    for (uint32_t kt = 0; kt < nK; ++kt) {
        const int buf = kt & 1;
        // Next tile's loads go out now; its split and LDS writes are spread over
        // the second half of this tile's K-slices so they overlap the MFMAs.
        // On the last tile the last tile is fetched again into the idle buffer.
        fetch(kt + 1 < nK ? kt + 1 : kt);
        // sign of this wave's rows against this K-tile from the bits above the tile
        const bool neg_tile = __popc((Pw >> 5) & ((kt * KT) >> 5)) & 1;
        const unsigned char* bbase = lds + buf * C::BUF + l32 * C::PITCH;
        bf16x8 Ap[2], An[2];
        if constexpr (PLANES == 3) {
            const uint32_t tm = neg_tile ? 0x80008000u : 0u;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                u32x4 p = {fA[e][0] ^ tm, fA[e][1] ^ tm, fA[e][2] ^ tm, fA[e][3] ^ tm};
                u32x4 n = p ^ 0x80008000u;
                Ap[e] = __builtin_bit_cast(bf16x8, p);
                An[e] = __builtin_bit_cast(bf16x8, n);
            }
        }
        const float ts = neg_tile ? -1.f : 1.f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if constexpr (PLANES == 3) {
                bf16x8 B[3][2];
#pragma unroll
                for (int pl = 0; pl < 3; ++pl)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        B[pl][cb] = *(const bf16x8*)(bbase + (pl * 2 + cb) * XT * C::PITCH + (16 * s + 8 * h) * 2);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const bool neg = popc_const((uint32_t)rb & (uint32_t)(s >> 1)) & 1;
                    const bf16x8 A = neg ? An[s & 1] : Ap[s & 1];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) {
                        acc[0][rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B[0][cb], acc[0][rb][cb], 0, 0, 0);
                        acc[ACC - 1][rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B[1][cb], acc[ACC - 1][rb][cb], 0, 0, 0);
                        acc[ACC - 1][rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B[2][cb], acc[ACC - 1][rb][cb], 0, 0, 0);
                    }
                }
            } else {
                f32x4 B[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    B[cb] = *(const f32x4*)(bbase + cb * XT * C::PITCH + (8 * s + 4 * h) * 4);
#pragma unroll
                for (int st = 0; st < 4; ++st) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const bool neg = popc_const((uint32_t)rb & (uint32_t)(s >> 2)) & 1;
                        const float A = (neg ? -ts : ts) * fF[s & 3][st];
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[0][rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B[cb][st], acc[0][rb][cb], 0, 0, 0);
                    }
                }
            }
            // deposit pieces scheduled after this slice
            int nparts = 0;
#pragma unroll
            for (int part = 0; part < NPARTS; ++part) {
                constexpr int H0 = S / 2;
                const int sp = H0 + part * (S - H0) / NPARTS;
                if (sp == s) {
                    deposit_part(buf ^ 1, part / 4, part % 4);
                    ++nparts;
                }
            }
            // Scheduling: this slice's LDS reads first, then its MFMAs with the
            // split arithmetic of the deposit pieces threaded between them, then
            // the pieces' LDS writes.
            constexpr int MF = PLANES == 3 ? RB * 6 : RB * 8;   // MFMAs per slice
            __builtin_amdgcn_sched_group_barrier(0x100, PLANES == 3 ? 6 : 2, 0);
            if (nparts > 0) {
#pragma unroll
                for (int i = 0; i < MF; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, PLANES == 3 ? 6 : 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x200, 16, 0);
            } else {
                __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);
            }
        }
        __syncthreads();
    }

    // ---- epilogue: binary64 recombination, phase, scale, staged store ----
    const double scale = prm.scale;
    const int esz = prm.out128 ? 16 : 8;
    unsigned char* stage = lds + wave * 1024 * esz;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const uint32_t pb = Pw + 32 * rb;   // first row of this 32x32 block
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t pl = 8 * (r >> 2) + 4 * h + (r & 3);
            double re = (double)acc[0][rb][0][r];
            double im = (double)acc[0][rb][1][r];
            if constexpr (ACC == 2) {
                re += (double)acc[ACC - 1][rb][0][r];
                im += (double)acc[ACC - 1][rb][1][r];
            }
            re *= scale;
            im *= scale;
            uint32_t slot;
            if constexpr (DIR == FORWARD) {
                rotate_minus_i(re, im, (uint32_t)__popc((X0 + l32) & (pb + pl)));
                slot = pauli_index((uint32_t)l32, pl);           // offset inside the 1024-run
            } else {
                slot = ((pl ^ (uint32_t)l32) << 5) | pl;        // (row, col) inside the 32x32 square
            }
            if (prm.out128) *(double2*)(stage + slot * 16) = make_double2(re, im);
            else *(float2*)(stage + slot * 8) = make_float2((float)re, (float)im);
        }
        __syncthreads();
        if constexpr (DIR == FORWARD) {
            // contiguous run of min(1024, 4^N) coefficients starting at n(X0, pb)
            const uint32_t run = D < 32u ? D * D : 1024u;
            unsigned char* o = dst + (size_t)pauli_index(X0, pb) * esz;
            if (pb < D) {
                if (run * esz >= 16) {
                    for (uint32_t b = lane * 16; b < run * esz; b += 64 * 16)
                        *(u32x4*)(o + b) = *(const u32x4*)(stage + b);
                } else if (lane == 0) {
                    *(u32x2*)o = *(const u32x2*)stage;   // N = 0, binary32 output
                }
            }
        } else {
            // 32x32 square of G: rows (pb ^ X0) + rl, columns pb + cl
            const uint32_t w = D < 32u ? D : 32u;
            const uint32_t rowbytes = w * esz;
            const uint32_t r0 = (pb ^ X0) & ~31u;
            if (rowbytes >= 16) {
                for (uint32_t b = lane * 16; b < w * rowbytes; b += 64 * 16) {
                    const uint32_t rl = b / rowbytes, cb = b % rowbytes;
                    if (pb < D)
                        *(u32x4*)(dst + ((size_t)(r0 + rl) * D + pb) * esz + cb) =
                            *(const u32x4*)(stage + rl * 32 * esz + cb);
                }
            } else if (lane == 0) {
                *(u32x2*)dst = *(const u32x2*)stage;     // N = 0, binary32 output
            }
        }
        __syncthreads();
    }
}

// ---- tile table ----
struct TileDesc {
    int rb, waves;
};
constexpr TileDesc TILES[] = {
    {4, 4},  // 1: 512 rows x 32 x, K-tile 128
    {2, 4},  // 2: 256 rows, K-tile 64
    {2, 8},  // 3: 512 rows, K-tile 64
    {1, 4},  // 4: 128 rows, K-tile 32
    {1, 1},  // 5: 32 rows, K-tile 32 (zero-padded below 32)
    {1, 2},  // 6: 64 rows, K-tile 32
};
constexpr int NTILES = sizeof(TILES) / sizeof(TILES[0]);

template <int PLANES, int RB, int WAVES, int DIR>
hipError_t launch_cfg(const Params& p, bool in128, int batch, hipStream_t s) {
    using C = Cfg<PLANES, RB, WAVES>;
    const uint32_t D = 1u << p.N;
    const uint32_t nMB = D > (uint32_t)C::MT ? D / C::MT : 1u;
    const uint32_t nXB = D > (uint32_t)XT ? D / XT : 1u;
    auto kern = in128 ? mfma_kernel<PLANES, RB, WAVES, DIR, true> : mfma_kernel<PLANES, RB, WAVES, DIR, false>;
    const int lds = C::lds_bytes(p.out128 ? 16 : 8);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nMB * nXB, batch), dim3(WAVES * 64), lds, s, p);
    return hipGetLastError();
}

template <int PLANES, int DIR>
hipError_t launch_tile(int tile, const Params& p, bool in128, int batch, hipStream_t s) {
    switch (tile) {
        case 1: return launch_cfg<PLANES, 4, 4, DIR>(p, in128, batch, s);
        case 2: return launch_cfg<PLANES, 2, 4, DIR>(p, in128, batch, s);
        case 3: return launch_cfg<PLANES, 2, 8, DIR>(p, in128, batch, s);
        case 4: return launch_cfg<PLANES, 1, 4, DIR>(p, in128, batch, s);
        case 5: return launch_cfg<PLANES, 1, 1, DIR>(p, in128, batch, s);
        case 6: return launch_cfg<PLANES, 1, 2, DIR>(p, in128, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int mfma_tile_count(int /*planes*/) { return NTILES; }

bool mfma_tile_valid(int /*planes*/, int tile, int N) {
    if (tile < 1 || tile > NTILES) return false;
    const TileDesc t = TILES[tile - 1];
    const uint32_t D = 1u << N;
    if (t.rb == 1 && t.waves == 1) return true;       // pads any N up to 32
    return D >= (uint32_t)(t.rb * t.waves * 32);      // full row and K tiles
}

int mfma_default_tile(int planes, int N) {
    (void)planes;
    if (N >= 9) return 1;
    if (N == 8) return 2;
    if (N == 7) return 4;
    if (N == 6) return 6;
    return 5;
}

hipError_t launch_mfma(Dir dir, int planes, const void* in, bool in_c128, void* out,
                       bool out_c128, int N, int batch, double scale, int tile,
                       hipStream_t stream) {
    if (tile == 0) tile = mfma_default_tile(planes, N);
    if (!mfma_tile_valid(planes, tile, N)) return hipErrorInvalidValue;
    Params p{in, out, N, out_c128 ? 1 : 0, scale};
    if (planes == 3)
        return dir == FORWARD ? launch_tile<3, FORWARD>(tile, p, in_c128, batch, stream)
                              : launch_tile<3, ADJOINT>(tile, p, in_c128, batch, stream);
    return dir == FORWARD ? launch_tile<1, FORWARD>(tile, p, in_c128, batch, stream)
                          : launch_tile<1, ADJOINT>(tile, p, in_c128, batch, stream);
}

}  // namespace pauli
