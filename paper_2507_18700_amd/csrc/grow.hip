// Adaptive growth of the hidden width (Sec. II B, Fig. 2(b)): every parameter
// of the smaller model is copied to its place in the larger one, every new
// entry is a fresh N(0, eps^2) draw, and the Adam moments are zero-padded
// (App. B).  One thread per destination entry.
#include "kernels.h"

namespace vmc {

// Source index of destination entry e of the grown model, or -1 if e is new.
// New hidden units are appended at the end of each h-block; one-hot columns
// keep their order.
__device__ inline int64_t grow_source(int dims, int d0, int d1, int glu, int cplx, int64_t e) {
    ParamLayout A = param_layout(dims, d0, glu, cplx), B = param_layout(dims, d1, glu, cplx);
    auto mat = [&](int64_t b0, int64_t b1, int rows0, int rows1, int cols1, int kind, int64_t &src) -> bool {
        // kind: 0 plain [rows][d], 1 = 1D gate [h;x], 2 = 2D gate [hz;hv;x], 3 = 2D U [hz;hv],
        //       4 = fixed columns (W_in: 2), 5 = bias vector, 6 = head rows [2][d]
        int64_t n1 = (int64_t)rows1 * cols1;
        if (e < b1 || e >= b1 + n1) return false;
        int64_t rel = e - b1;
        int row = (int)(rel / cols1), c = (int)(rel % cols1);
        src = -1;
        if (row >= rows0) return true;
        int cols0, c0 = -1;
        switch (kind) {
            case 0: cols0 = d0; c0 = c < d0 ? c : -1; break;
            case 1: cols0 = d0 + 2; c0 = c < d1 ? (c < d0 ? c : -1) : d0 + (c - d1); break;
            case 2:
                cols0 = 2 * d0 + 4;
                if (c < d1) c0 = c < d0 ? c : -1;
                else if (c < 2 * d1) c0 = (c - d1) < d0 ? d0 + (c - d1) : -1;
                else c0 = 2 * d0 + (c - 2 * d1);
                break;
            case 3:
                cols0 = 2 * d0;
                if (c < d1) c0 = c < d0 ? c : -1;
                else c0 = (c - d1) < d0 ? d0 + (c - d1) : -1;
                break;
            case 4: cols0 = cols1; c0 = c; break;
            case 6: cols0 = d0; c0 = c < d0 ? c : -1; break;
            default: cols0 = 1; c0 = 0; break;
        }
        if (c0 >= 0) src = b0 + (int64_t)row * cols0 + c0;
        return true;
    };
    int64_t src = -1;
    if (dims == 1) {
        if (mat(A.Wg, B.Wg, d0, d1, d1 + 2, 1, src)) return src;
        if (mat(A.bg, B.bg, d0, d1, 1, 5, src)) return src;
        if (mat(A.Wr, B.Wr, d0, d1, d1 + 2, 1, src)) return src;
        if (mat(A.br, B.br, d0, d1, 1, 5, src)) return src;
        if (mat(A.Wh, B.Wh, d0, d1, d1, 0, src)) return src;
        if (mat(A.bh, B.bh, d0, d1, 1, 5, src)) return src;
        if (mat(A.Win, B.Win, d0, d1, 2, 4, src)) return src;
        if (mat(A.bin, B.bin, d0, d1, 1, 5, src)) return src;
    } else {
        if (mat(A.W, B.W, d0, d1, 2 * d1 + 4, 2, src)) return src;
        if (mat(A.b, B.b, d0, d1, 1, 5, src)) return src;
        if (mat(A.Wg, B.Wg, d0, d1, 2 * d1 + 4, 2, src)) return src;
        if (mat(A.bg, B.bg, d0, d1, 1, 5, src)) return src;
        if (mat(A.U, B.U, d0, d1, 2 * d1, 3, src)) return src;
    }
    if (glu) {
        if (mat(A.W1, B.W1, d0, d1, d1, 0, src)) return src;
        if (mat(A.b1, B.b1, d0, d1, 1, 5, src)) return src;
        if (mat(A.W2, B.W2, d0, d1, d1, 0, src)) return src;
        if (mat(A.b2, B.b2, d0, d1, 1, 5, src)) return src;
    }
    if (mat(A.Ua, B.Ua, 2, 2, d1, 6, src)) return src;
    if (mat(A.ca, B.ca, 2, 2, 1, 5, src)) return src;
    if (cplx) {
        if (mat(A.Up, B.Up, 2, 2, d1, 6, src)) return src;
        if (mat(A.cp, B.cp, 2, 2, 1, 5, src)) return src;
    }
    return -1;
}

__global__ void grow_kernel(int dims, int d0, int d1, int glu, int cplx, int64_t n_to, const float *p0,
                            uint64_t seed, double noise, float *p1, const float *m0, const float *v0,
                            float *m1, float *v1) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_to;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t src = grow_source(dims, d0, d1, glu, cplx, e);
        if (src >= 0) {
            p1[e] = p0[src];
            if (m1) {
                m1[e] = m0[src];
                v1[e] = v0[src];
            }
        } else {
            // Box-Muller on two 24-bit Philox uniforms keyed by (seed, e)
            uint32_t c[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0u, 0u};
            philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
            double u1 = ((double)(c[0] >> 8) + 1.0) * (1.0 / 16777216.0);
            double u2 = (double)(c[1] >> 8) * (1.0 / 16777216.0);
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925287 * u2);
            p1[e] = (float)(noise * z);
            if (m1) {
                m1[e] = 0.0f;
                v1[e] = 0.0f;
            }
        }
    }
}

hipError_t launch_grow(const vmc_model &from, const float *p0, int new_dh, uint64_t seed, double noise,
                       float *p1, const float *m0, const float *v0, float *m1, float *v1, int64_t n_to,
                       hipStream_t st) {
    int grid = (int)((n_to + 255) / 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(grow_kernel, dim3(grid), dim3(256), 0, st, from.dims, from.d_h, new_dh, from.glu,
                       from.is_complex, n_to, p0, seed, noise, p1, m0, v0, m1, v1);
    return hipGetLastError();
}

// Fill kernel (used instead of memset so that calls can sit in a captured graph).
__global__ void fill_f32(float *p, int64_t n, float v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st) {
    int grid = (int)((n + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fill_f32, dim3(grid), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace vmc
