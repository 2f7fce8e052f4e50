// Shared device/host helpers of libpauli (gfx950).
//
// Index conventions (T. Jones 2024, section 2): a Pauli string n is split
// into a flip mask x (bit t set for X or Y on qubit t) and a phase mask z
// (bit t set for Y or Z).  With operator flag_t = 2*bit(2t+1) + bit(2t)
// (0=I, 1=X, 2=Y, 3=Z) this gives x_t = bit(2t) ^ bit(2t+1), z_t = bit(2t+1),
// and back n = spread_even(x ^ z) | spread_odd(z).  The coefficient is
//   c(x,z) = 2^-N (-i)^{popc(x&z)} sum_i (-1)^{popc(i&z)} G[i^x][i]
// (Eq. (c_def_in_terms_of_fn) with lambda of Eq. (lambda_def) written out
// for the Pauli matrices of Eq. (3)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pauli {

// Spread the low 16 bits of v to the even bit positions of a 32-bit word.
__host__ __device__ inline uint32_t spread_even(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Gather the even bits of v into the low 16 bits.
__host__ __device__ inline uint32_t compact_even(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

// Coefficient index of the string with flip mask x and phase mask z.
__host__ __device__ inline uint32_t pauli_index(uint32_t x, uint32_t z) {
    return spread_even(x ^ z) | (spread_even(z) << 1);
}

__host__ __device__ inline uint32_t flip_of_index(uint32_t n) {
    return compact_even(n) ^ compact_even(n >> 1);
}

__host__ __device__ inline uint32_t phase_of_index(uint32_t n) { return compact_even(n >> 1); }

// Inverse Gray code: position k with k ^ (k >> 1) == g (prefix XOR).
__host__ __device__ inline uint32_t gray_inverse(uint32_t g) {
    g ^= g >> 16;
    g ^= g >> 8;
    g ^= g >> 4;
    g ^= g >> 2;
    g ^= g >> 1;
    return g;
}

__host__ __device__ constexpr uint32_t gray(uint32_t k) { return k ^ (k >> 1); }

__host__ __device__ constexpr int popc_const(uint32_t v) {
    return v == 0 ? 0 : (int)(v & 1u) + popc_const(v >> 1);
}

// Multiply (re, im) by (-i)^k  (k taken mod 4); exact.
template <typename T>
__device__ inline void rotate_minus_i(T& re, T& im, uint32_t k) {
    T r = re, m = im;
    switch (k & 3u) {
        case 0: break;
        case 1: re = m; im = -r; break;   // -i (r + i m) = m - i r
        case 2: re = -r; im = -m; break;
        default: re = -m; im = r; break;  // i (r + i m) = -m + i r
    }
}

// Blocks with consecutive logical ids share input slabs; the hardware hands
// consecutive workgroup ids to the 8 XCDs round-robin, so remap them to give
// each XCD a contiguous range of logical ids (its own slabs, in its own L2).
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t total) {
    if ((total & 7u) != 0u) return b;
    return (b & 7u) * (total >> 3) + (b >> 3);
}

}  // namespace pauli
