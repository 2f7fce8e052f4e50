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
// Precision.  PLANES = 3: each binary32 component g is split exactly as
// g = hi + mid + lo with hi = bf16(g), mid = bf16(g - hi), lo = g - hi - mid
// (exact in bf16 for normal g); bf16 MFMA accumulates hi into one FP32
// accumulator and mid + lo into a second, and the two are added in binary64
// in the epilogue before the phase and scale.  PLANES = 1: binary32 MFMA on
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

// Exact three-way bf16 split of two binary32 values (round-to-nearest-even).
__device__ inline void split3(float a, float b, uint32_t& h, uint32_t& m, uint32_t& l) {
    h = pack_bf16(a, b);
    const float ra = a - lo_half(h), rb = b - hi_half(h);
    m = pack_bf16(ra, rb);
    const float qa = ra - lo_half(m), qb = rb - hi_half(m);
    l = pack_bf16(qa, qb);
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
    int in128;
    int out128;
    double scale;
};

__device__ inline f32x2 load_elem(const void* base, size_t idx, int is128) {
    if (is128) {
        const double2 v = ((const double2*)base)[idx];
        return f32x2{(float)v.x, (float)v.y};
    }
    const float2 v = ((const float2*)base)[idx];
    return f32x2{v.x, v.y};
}

template <int PLANES, int RB, int WAVES, int DIR>
__global__ __launch_bounds__(WAVES * 64) void mfma_kernel(Params prm) {
    using C = Cfg<PLANES, RB, WAVES>;
    constexpr int KT = C::KT;
    constexpr int ACC = PLANES == 3 ? 2 : 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

    const int N = prm.N;
    const uint32_t D = 1u << N;
    const uint32_t nMB = D > (uint32_t)C::MT ? D / C::MT : 1u;   // row blocks
    const uint32_t nK = D > (uint32_t)KT ? D / KT : 1u;          // K tiles
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const uint32_t xb = L / nMB, mb = L % nMB;
    const uint32_t X0 = xb * XT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const uint32_t Pw = mb * C::MT + wave * RB * 32;            // first row of this wave
    const size_t mat = (size_t)D * D;
    const unsigned char* src = (const unsigned char*)prm.in + (size_t)blockIdx.y * mat * (prm.in128 ? 16 : 8);
    unsigned char* dst = (unsigned char*)prm.out + (size_t)blockIdx.y * mat * (prm.out128 ? 16 : 8);

    // ---- prologue: fetch one K-tile (registers) and deposit it (LDS) ----
    f32x2 stg[C::UPT][16];
    auto fetch = [&](uint32_t kt) {
        const uint32_t Q0 = kt * KT;
#pragma unroll
        for (int u = 0; u < C::UPT; ++u) {
            const int ub = tid + u * C::NT;
            if (ub >= C::UBLK) break;
            const int g = ub >> 6, w6 = ub & 63;   // 32x32 square g of the tile, block w6 in it
            if (DIR == FORWARD) {
                const int mr = w6 >> 3, mc = w6 & 7;
                const uint32_t q0 = Q0 + 32 * g + 4 * mc;
                const uint32_t r0 = ((Q0 + 32 * g) ^ X0) & ~31u;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const uint32_t r = r0 + 4 * mr + a;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t q = q0 + b;
                        stg[u][a * 4 + b] = (r < D && q < D) ? load_elem(src, (size_t)r * D + q, prm.in128)
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
                    f32x2 v = {0.f, 0.f};
                    if (z < D && x < D) {
                        const f32x2 c = load_elem(src, nb + o, prm.in128);
                        float re = c.x, im = c.y;
                        rotate_minus_i(re, im, 3u * (uint32_t)__popc(x & z));  // i^{popc}
                        v = f32x2{re, im};
                    }
                    stg[u][r] = v;
                }
            }
        }
    };
    auto deposit = [&](int buf) {
        unsigned char* base = lds + buf * C::BUF;
#pragma unroll
        for (int u = 0; u < C::UPT; ++u) {
            const int ub = tid + u * C::NT;
            if (ub >= C::UBLK) break;
            const int g = ub >> 6, w6 = ub & 63;
            int xh, kh;  // micro-block column group (x_l / 4) and first K slot
            if (DIR == FORWARD) {
                const int mr = w6 >> 3, mc = w6 & 7;
                xh = mr ^ mc;
                kh = 32 * g + 4 * mc;
            } else {
                // 16 consecutive coefficients: o = 16*w6 + r, r = (x^z)_0 | z_0<<1 | (x^z)_1<<2 | z_1<<3
                const uint32_t o = 16 * w6;
                const int zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
                xh = xl >> 2;
                kh = 32 * g + zl;
            }
#pragma unroll
            for (int x2 = 0; x2 < 4; ++x2) {
                f32x2 e[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (DIR == FORWARD) {
                        e[b] = stg[u][((x2 ^ b) << 2) | b];  // row a = x2 ^ b, column b
                    } else {
                        const int d = x2 ^ b;                 // (x ^ z) low bits
                        e[b] = stg[u][(d & 1) | ((b & 1) << 1) | ((d >> 1) << 2) | ((b >> 1) << 3)];
                    }
                }
                const int col = xh * 4 + x2;
                unsigned char* cbase = base + col * C::PITCH + kh * C::ESZ;
                if constexpr (PLANES == 3) {
                    uint32_t hr0, mr0, lr0, hr1, mr1, lr1, hi0, mi0, li0, hi1, mi1, li1;
                    split3(e[0].x, e[1].x, hr0, mr0, lr0);
                    split3(e[2].x, e[3].x, hr1, mr1, lr1);
                    split3(e[0].y, e[1].y, hi0, mi0, li0);
                    split3(e[2].y, e[3].y, hi1, mi1, li1);
                    constexpr int PS = XT * C::PITCH;  // plane stride
                    *(u32x2*)(cbase + 0 * PS) = u32x2{hr0, hr1};
                    *(u32x2*)(cbase + 1 * PS) = u32x2{hi0, hi1};
                    *(u32x2*)(cbase + 2 * PS) = u32x2{mr0, mr1};
                    *(u32x2*)(cbase + 3 * PS) = u32x2{mi0, mi1};
                    *(u32x2*)(cbase + 4 * PS) = u32x2{lr0, lr1};
                    *(u32x2*)(cbase + 5 * PS) = u32x2{li0, li1};
                } else {
                    constexpr int PS = XT * C::PITCH;
                    *(f32x4*)(cbase) = f32x4{e[0].x, e[1].x, e[2].x, e[3].x};
                    *(f32x4*)(cbase + PS) = f32x4{e[0].y, e[1].y, e[2].y, e[3].y};
                }
            }
        }
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
    deposit(0);
    __syncthreads();
    for (uint32_t kt = 0; kt < nK; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nK) fetch(kt + 1);
        // sign of this wave's rows against this K-tile from the bits above the tile
        const bool neg_tile = __popc((Pw >> 5) & ((kt * KT) >> 5)) & 1;
        const unsigned char* bbase = lds + buf * C::BUF + l32 * C::PITCH;
        if constexpr (PLANES == 3) {
            const uint32_t tm = neg_tile ? 0x80008000u : 0u;
            bf16x8 Ap[2], An[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                u32x4 p = {fA[e][0] ^ tm, fA[e][1] ^ tm, fA[e][2] ^ tm, fA[e][3] ^ tm};
                u32x4 n = p ^ 0x80008000u;
                Ap[e] = __builtin_bit_cast(bf16x8, p);
                An[e] = __builtin_bit_cast(bf16x8, n);
            }
#pragma unroll
            for (int s = 0; s < KT / 16; ++s) {
                bf16x8 B[3][2];
#pragma unroll
                for (int pl = 0; pl < 3; ++pl)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        B[pl][cb] = *(const bf16x8*)(bbase + (pl * 2 + cb) * XT * C::PITCH +
                                                     (16 * s + 8 * h) * 2);
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
            }
        } else {
            const float ts = neg_tile ? -1.f : 1.f;
#pragma unroll
            for (int s = 0; s < KT / 8; ++s) {
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
        }
        if (kt + 1 < nK) deposit(buf ^ 1);
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
            if (DIR == FORWARD) {
                rotate_minus_i(re, im, (uint32_t)__popc((X0 + l32) & (pb + pl)));
                slot = pauli_index((uint32_t)l32, pl);           // offset inside the 1024-run
            } else {
                slot = ((pl ^ (uint32_t)l32) << 5) | pl;        // (row, col) inside the 32x32 square
            }
            if (prm.out128) *(double2*)(stage + slot * 16) = make_double2(re, im);
            else *(float2*)(stage + slot * 8) = make_float2((float)re, (float)im);
        }
        __syncthreads();
        if (DIR == FORWARD) {
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
hipError_t launch_cfg(const Params& p, int batch, hipStream_t s) {
    using C = Cfg<PLANES, RB, WAVES>;
    const uint32_t D = 1u << p.N;
    const uint32_t nMB = D > (uint32_t)C::MT ? D / C::MT : 1u;
    const uint32_t nXB = D > (uint32_t)XT ? D / XT : 1u;
    auto kern = mfma_kernel<PLANES, RB, WAVES, DIR>;
    const int lds = C::lds_bytes(p.out128 ? 16 : 8);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nMB * nXB, batch), dim3(WAVES * 64), lds, s, p);
    return hipGetLastError();
}

template <int PLANES, int DIR>
hipError_t launch_tile(int tile, const Params& p, int batch, hipStream_t s) {
    switch (tile) {
        case 1: return launch_cfg<PLANES, 4, 4, DIR>(p, batch, s);
        case 2: return launch_cfg<PLANES, 2, 4, DIR>(p, batch, s);
        case 3: return launch_cfg<PLANES, 2, 8, DIR>(p, batch, s);
        case 4: return launch_cfg<PLANES, 1, 4, DIR>(p, batch, s);
        case 5: return launch_cfg<PLANES, 1, 1, DIR>(p, batch, s);
        case 6: return launch_cfg<PLANES, 1, 2, DIR>(p, batch, s);
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
    Params p{in, out, N, in_c128 ? 1 : 0, out_c128 ? 1 : 0, scale};
    if (planes == 3)
        return dir == FORWARD ? launch_tile<3, FORWARD>(tile, p, batch, stream)
                              : launch_tile<3, ADJOINT>(tile, p, batch, stream);
    return dir == FORWARD ? launch_tile<1, FORWARD>(tile, p, batch, stream)
                          : launch_tile<1, ADJOINT>(tile, p, batch, stream);
}

}  // namespace pauli
