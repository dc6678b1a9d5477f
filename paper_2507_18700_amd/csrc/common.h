// Device-side building blocks shared by the gfx950 kernels of the library:
// MFMA fragment types, bfloat16 conversion, activations, Philox, the lattice
// order of the autoregressive chain and the workspace/staging layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vmcrnn.h"

namespace vmc {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4_t;
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// two floats to packed bfloat16 (round to nearest even), one v_cvt_pk_bf16_f32
__device__ inline uint32_t pack_bf16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

constexpr int WAVE = 64;
constexpr float PI_F = 3.14159265358979323846f;

// ---------------------------------------------------------------- precision
// Storage tags of the contraction operands.  Both use 16-byte fragments per
// lane: lane l of a 16x16 MFMA tile supplies row (l % 16) and the VEC
// consecutive contraction indices starting at VEC * (l / 16) of a KSTEP-wide
// slice.  For FP32 the four floats of a fragment feed four 16x16x4 MFMAs whose
// contraction index sets interleave; the same interleave is used for both
// operands, so the sum is unchanged.
struct F32 {
    typedef float store_t;
    static constexpr int VEC = 4;
    static constexpr int KSTEP = 16;
    __device__ static inline store_t from_float(float x) { return x; }
    __device__ static inline float to_float(store_t x) { return x; }
    __device__ static inline void mma(f32x4_t &acc, const uint4 &a, const uint4 &b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
    }
};

// bfloat16 from float, round to nearest even (NaN stays NaN).
__host__ __device__ inline uint16_t f2bf(float x) {
    uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
    u = __float_as_uint(x);
#else
    __builtin_memcpy(&u, &x, 4);
#endif
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

struct BF16 {
    typedef uint16_t store_t;
    static constexpr int VEC = 8;
    static constexpr int KSTEP = 32;
    __device__ static inline store_t from_float(float x) { return f2bf(x); }
    __device__ static inline float to_float(store_t x) { return bf2f(x); }
    __device__ static inline void mma(f32x4_t &acc, const uint4 &a, const uint4 &b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                      __builtin_bit_cast(bf16x8_t, b), acc, 0, 0, 0);
    }
};

// -------------------------------------------------------------- activations
// Logistic function and tanh from the hardware exp2 (v_exp_f32) and
// reciprocal (v_rcp_f32, 1 ulp); tanh via 2*sigmoid(2x) - 1, whose absolute
// error stays at float rounding level.
__device__ inline float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float sigmoidf_(float x) {
    return rcpf_(1.0f + __builtin_amdgcn_exp2f(x * -1.4426950408889634f));  // -log2(e)
}
__device__ inline float tanhf_(float x) {
    return 2.0f * rcpf_(1.0f + __builtin_amdgcn_exp2f(x * -2.8853900817779268f)) - 1.0f;  // -2 log2(e)
}
__device__ inline float softsignf_(float x) { return x / (1.0f + fabsf(x)); }

// ------------------------------------------------------------------- Philox
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ------------------------------------------------------------ chain order
// Order position n -> lattice site of the zig-zag path (1D: identity).
__host__ __device__ inline int order_site(int n, int Lx) {
    int j = n / Lx, k = n - j * Lx;
    return j * Lx + ((j & 1) ? (Lx - 1 - k) : k);
}
__host__ __device__ inline int site_pos(int site, int Lx) {
    int j = site / Lx, i = site - j * Lx;
    return j * Lx + ((j & 1) ? (Lx - 1 - i) : i);
}

// --------------------------------------------------------- staged weights
// Device copy of the parameters in MFMA-ready form, padded to DH (a multiple
// of 16 >= d_h) with zeros, built by the staging kernel for every call (the
// exact layouts are documented at stage_weights):
//   Bc  cell weights, row n = gate*DH + unit; 1D gates (u, r, m) = (W_g, W_r,
//       W_h) on h_{n-1}; 2D gates (c, u, v) = (W, W_g, U) on [h_hz | h_vt];
//       followed by the one-hot (indicator) columns;  BcT its hidden part
//       transposed (backward);  Bg / BgT the GLU (W_1 rows, then W_2 rows).
//   E   [ESLOTS][DH] FP32 epilogue table, see the slot names below.
//   Hd  [4][DH]     heads U_a (rows 0,1) and U_p (rows 2,3); hc[4]: c_a, c_p.
enum {
    // 1D
    E1_BG = 0, E1_XG0, E1_XG1, E1_BR, E1_XR0, E1_XR1, E1_BH, E1_BIN, E1_XIN0, E1_XIN1,
    // 2D
    E2_B = 0, E2_XH0, E2_XH1, E2_XV0, E2_XV1, E2_BG, E2_XGH0, E2_XGH1, E2_XGV0, E2_XGV1,
    // both
    E_B1 = 10, E_B2 = 11, ESLOTS = 12
};

struct Dims {
    int dims, Lx, Ly, N, dh, DH, K, KP, cplx, glu, prec;
    // launch choices from the tuning table (host side): the alternative row
    // tile, persistent work-groups per compute unit of the suffix-chain launch
    int row_alt, chain_wpc;
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Source offsets of the flat parameter vector (the layout in vmcrnn.h).
struct ParamLayout {
    int64_t Wg, bg, Wr, br, Wh, bh, Win, bin;  // 1D
    int64_t W, b, U;                           // 2D (Wg, bg shared)
    int64_t W1, b1, W2, b2, Ua, ca, Up, cp, total;
};

__host__ __device__ inline ParamLayout param_layout(int dims, int d, int glu, int cplx) {
    ParamLayout L = {};
    int64_t o = 0;
    if (dims == 1) {
        L.Wg = o; o += (int64_t)d * (d + 2);
        L.bg = o; o += d;
        L.Wr = o; o += (int64_t)d * (d + 2);
        L.br = o; o += d;
        L.Wh = o; o += (int64_t)d * d;
        L.bh = o; o += d;
        L.Win = o; o += (int64_t)d * 2;
        L.bin = o; o += d;
    } else {
        L.W = o; o += (int64_t)d * (2 * d + 4);
        L.b = o; o += d;
        L.Wg = o; o += (int64_t)d * (2 * d + 4);
        L.bg = o; o += d;
        L.U = o; o += (int64_t)d * 2 * d;
    }
    if (glu) {
        L.W1 = o; o += (int64_t)d * d;
        L.b1 = o; o += d;
        L.W2 = o; o += (int64_t)d * d;
        L.b2 = o; o += d;
    }
    L.Ua = o; o += 2 * d;
    L.ca = o; o += 2;
    if (cplx) {
        L.Up = o; o += 2 * d;
        L.cp = o; o += 2;
    }
    L.total = o;
    return L;
}

}  // namespace vmc
