// Shared device helpers of the gfx950 ICM library: complex type, Philox
// counter-based generator, Box-Muller normals and the Peskin kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "normal64.h"

namespace icm {

// Global-memory pointers. Pointers read from a device-resident descriptor are
// generic to the compiler and would be accessed with flat instructions, which
// also count against the LDS wait counter; converting them once gives plain
// global loads and stores.
// (The host pass only checks kernel bodies, so there they are plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
    return (gptr<T>)p;
}

template <typename T>
struct cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }
// multiply by i (s = +1) or -i (s = -1)
template <typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a, int s) {
    return s > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------- Philox
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// multiplies counter words 0 and 2 by fixed odd constants, and mixes the
// high/low halves of the products with words 1 and 3 and the round key; the
// key advances by the Weyl constants between rounds.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit multiply (v_mad_u64_u32) per product gives
        // both halves at once
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // each three-input xor is one gfx950 bitop3 (truth table 0x96)
        const uint32_t x0 = (uint32_t)__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96);
        const uint32_t x2 = (uint32_t)__builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96);
        c = u32x4{x0, lo1, x2, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Counter layout: (index, step mod 2^32, (replica << 4) | block, step >> 32),
// key (seed mod 2^32, seed >> 32). The stochastic stress uses the index of a
// z pair of cells and blocks 0-2; the equilibrium sample the cell index and
// block 3.
struct NoiseKey {
    uint32_t k0, k1;      // seed words
    uint32_t step_lo, step_hi;
    uint32_t rep_tag;     // replica << 4
};

__device__ __forceinline__ u32x4 noise_words(const NoiseKey& nk, uint32_t index, uint32_t block) {
    return philox4x32_10(u32x4{index, nk.step_lo, nk.rep_tag | block, nk.step_hi}, nk.k0, nk.k1);
}

// Box-Muller: first word -> radius via u1 = (w+1) 2^-32 in (0,1], second word
// -> angle 2 pi u2 with u2 = w 2^-32 in [0,1). The FP64 transform takes the
// logarithm table of normal64.h, kept in the calling kernel's LDS and filled
// by fill_log_tab before its first use.
struct LogTab {
    const double* inv;
    const double* lnf;
};

__device__ __forceinline__ void fill_log_tab(double* inv, double* lnf) {
    for (int j = threadIdx.x; j < kLogTab; j += blockDim.x) log_table_entry(j, inv, lnf);
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1, const LogTab& lt) {
    box_muller64(wa, wb, lt.inv, lt.lnf, z0, z1);
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1, const LogTab&) {
    // FP32 transform of the same words with the hardware log2, square root
    // (-2 ln u1 lies in [0, 44.4], no denormals) and sine/cosine, which take
    // their argument in revolutions.
    const float u1 = fmaf((float)wa, 2.3283064365386963e-10f, 2.3283064365386963e-10f);
    const float u2 = (float)wb * 2.3283064365386963e-10f;
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));  // (-2 ln u1)^(1/2)
    z0 = r * __builtin_amdgcn_cosf(u2);
    z1 = r * __builtin_amdgcn_sinf(u2);
}

// ---------------------------------------------------------- Peskin kernels
// Three-point kernel: minimal support with sum phi = 1, zero first moment and
// sum phi^2 = 1/2 (Sec. III.A.1); four-point kernel of Peskin (2002): support 4
// with the even/odd sums 1/2, zero first moment and sum phi^2 = 3/8.
__host__ __device__ __forceinline__ double phi3(double r) {
    const double s = fabs(r);
    if (s <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * s * s)) / 3.0;
    if (s <= 1.5) {
        const double t = 1.0 - s;
        return (5.0 - 3.0 * s - sqrt(fmax(1.0 - 3.0 * t * t, 0.0))) / 6.0;
    }
    return 0.0;
}
__device__ __forceinline__ double dphi3(double r) {
    const double s = fabs(r);
    if (s <= 0.5) return -r / sqrt(1.0 - 3.0 * r * r);
    if (s <= 1.5) {
        const double t = 1.0 - s;
        const double v = -0.5 - t / (2.0 * sqrt(fmax(1.0 - 3.0 * t * t, 1e-300)));
        return r >= 0.0 ? v : -v;
    }
    return 0.0;
}
__device__ __forceinline__ double phi4(double r) {
    const double s = fabs(r);
    if (s <= 1.0) return (3.0 - 2.0 * s + sqrt(1.0 + 4.0 * s - 4.0 * s * s)) * 0.125;
    if (s <= 2.0) return (5.0 - 2.0 * s - sqrt(fmax(-7.0 + 12.0 * s - 4.0 * s * s, 0.0))) * 0.125;
    return 0.0;
}
__device__ __forceinline__ double dphi4(double r) {
    const double s = fabs(r);
    double v;
    if (s <= 1.0)
        v = (-2.0 + (4.0 - 8.0 * s) / (2.0 * sqrt(1.0 + 4.0 * s - 4.0 * s * s))) * 0.125;
    else if (s <= 2.0)
        v = (-2.0 - (12.0 - 8.0 * s) / (2.0 * sqrt(fmax(-7.0 + 12.0 * s - 4.0 * s * s, 1e-300)))) * 0.125;
    else
        return 0.0;
    return r >= 0.0 ? v : -v;
}

// Nodes and weights of one axis. x: blob coordinate in grid units measured
// from node 0 of the component grid. 3-point: nodes round(x) + {-1,0,1};
// 4-point: floor(x) + {-1,0,1,2}. Node indices are wrapped into [0, n).
template <int P>
struct AxisStencil {
    int node[P];
    double w[P];
};

// Folds a coordinate into [0, n] (up to rounding at the ends), so that the
// stencil nodes are small integers in [-2, n + 2] that one conditional wrap
// brings into [0, n); positions are kept unwrapped and may lie many boxes
// away. The subtraction is exact (Sterbenz) except within rounding of 0.
__device__ __forceinline__ double fold_coord(double x, int n) {
    const double nd = (double)n;
    return x - nd * floor(x / nd);
}

__device__ __forceinline__ int wrap_node(int node, int n) {
    return node < 0 ? node + n : (node >= n ? node - n : node);
}

// Weight (and derivative) of the node at offset d for the P-node layout.
// P = 4 with hs > 0 is the split three-point kernel of Sec. III.A.2: the
// mean of phi3 shifted by -hs and +hs (hs = s / (2h)); its support
// |d| < 3/2 + hs lies inside the four nodes for s <= h.
template <int P>
__device__ __forceinline__ double kern_w(double d, double hs) {
    if (P == 3) return phi3(d);
    return hs > 0.0 ? 0.5 * (phi3(d - hs) + phi3(d + hs)) : phi4(d);
}
template <int P>
__device__ __forceinline__ double kern_dw(double d, double hs) {
    if (P == 3) return dphi3(d);
    return hs > 0.0 ? 0.5 * (dphi3(d - hs) + dphi3(d + hs)) : dphi4(d);
}

template <int P>
__device__ __forceinline__ void axis_stencil(double x, int n, bool deriv, double inv_h, double hs,
                                             AxisStencil<P>& st) {
    x = fold_coord(x, n);
    const int mi = (int)((P == 3) ? floor(x + 0.5) : floor(x));
#pragma unroll
    for (int a = 0; a < P; ++a) {
        const int node = mi - 1 + a;
        const double d = x - (double)node;
        st.node[a] = wrap_node(node, n);
        st.w[a] = deriv ? kern_dw<P>(d, hs) * inv_h : kern_w<P>(d, hs);
    }
}

// Node and weight of tap a (0 <= a < P) of one axis, without arrays (so a
// runtime tap index stays in registers).
template <int P>
__device__ __forceinline__ void axis_tap(double x, int n, int a, bool deriv, double inv_h, double hs, int& node,
                                         double& w) {
    x = fold_coord(x, n);
    const int nd = (int)((P == 3) ? floor(x + 0.5) : floor(x)) - 1 + a;
    const double d = x - (double)nd;
    node = wrap_node(nd, n);
    w = deriv ? kern_dw<P>(d, hs) * inv_h : kern_w<P>(d, hs);
}

__host__ __device__ __forceinline__ int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

}  // namespace icm
