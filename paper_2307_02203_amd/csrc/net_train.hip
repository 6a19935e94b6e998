// Training kernels of the learned dependence field (Sec. 4, Eq. 3; Sec. 4.3).
//
// One step over B vertex pairs runs the network row-wise: the R = 2B positions
// (all first endpoints, then all second endpoints) go through the grid lookup
// and the encoder, the two latents of a pair are multiplied, and the decoder
// gives Phi.  The mean L1 loss is differentiated by hand:
//   forward   grid gather -> [X W^T + b, ReLU] x2 -> X W3^T + b3 -> product
//             -> [X W^T + b, ReLU] x2 -> w6 . d2 + b6
//   adjoint   dY W (masked by the forward ReLU), dW += dY^T X, db += sum dY,
//             the product rule across the merge, FP32 atomic scatter into the
//             grid levels with the trilinear weights.
// Layer products run on MFMA 32x32x16 bf16 with FP32 accumulate: activations
// and weights are rounded to bf16 as they enter the MFMA; everything stored
// (activations, gradients, parameters, Adam moments) is FP32.
//
//  rows_mma_kernel  Y[rows][NOUT] = epilogue(X[rows][KIN] A^T), A staged once per
//                   workgroup in LDS in MFMA operand order (A = W forward,
//                   A = W^T for the data adjoint); 64 rows per wave and tile.
//  wgrad_kernel     dW[128][KIN] += G^T X over rows: 64-row tiles of G and X are
//                   transposed through LDS so both operands are row-contiguous.
#include "net.hpp"

namespace ndf {

constexpr int kThreads = 256;

struct GridOffs {
    int64_t off[2][kL];
};

__device__ __forceinline__ int64_t grid_off(const GridOffs &go, int e, int l) {
    const int64_t a = l == 0 ? go.off[0][0] : (l == 1 ? go.off[0][1] : (l == 2 ? go.off[0][2] : go.off[0][3]));
    const int64_t b = l == 0 ? go.off[1][0] : (l == 1 ? go.off[1][1] : (l == 2 ? go.off[1][2] : go.off[1][3]));
    return e ? b : a;
}

// ------------------------------------------------------------- helpers ----
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    // i-th output of SplitMix64 (Steele, Lea, Flood 2014) started from `seed`
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void fill_kernel(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void uniform_kernel(float *__restrict__ p, int64_t n, float a, uint64_t seed,
                               int64_t ctr0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double u = (double)(splitmix64_at(seed, (uint64_t)(ctr0 + i)) >> 11) * 0x1.0p-53;
        p[i] = (float)(a * (2.0 * u - 1.0));
    }
}

static unsigned gs_blocks(int64_t n) {
    int64_t b = ceil_div(n, kThreads);
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

__device__ __forceinline__ int64_t row_vertex(const int64_t *pairs, int64_t B, int64_t n) {
    return n < B ? pairs[2 * n] : pairs[2 * (n - B) + 1];
}

// Row n's position as continuous coordinates in [-1, 1]^3 when the pairs are
// given as positions pos[B][2][3] (the training pairs of Sec. 4.3).
__device__ __forceinline__ const float *row_pos(const float *pos, int64_t B, int64_t n) {
    return pos + 3 * (n < B ? 2 * n : 2 * (n - B) + 1);
}

// Trilinear corners of row n on level l: from its vertex index (pairs) or its
// continuous position (pos, when non-null); cells hashed on hashed levels.
__device__ __forceinline__ void row_corners(const GridGeom &g, int l, const int64_t *pairs,
                                            const float *pos, int64_t B, int64_t n, int idx[8],
                                            float w[8]) {
    int R[3];
    level_dims(g, l, R);
    const uint32_t hm = level_hmask(g, l);
    if (pos) {
        const float *p = row_pos(pos, B, n);
        const float pp[3] = {p[0], p[1], p[2]};
        corners_pos32<true>(R, pp, idx, w, hm);
    } else {
        int64_t v = row_vertex(pairs, B, n);
        const int64_t V = (int64_t)g.nx * g.ny * g.nz;
        v = v < 0 ? 0 : (v >= V ? V - 1 : v);  // out-of-range pairs are clamped
        corners_R32<true>(g, R, v, idx, w, hm);
    }
}

// ----------------------------------------------------------- grid fwd ----
// H0[n][l*8 + f] for rows n < 2B (first endpoints, then second endpoints).
__global__ __launch_bounds__(kThreads) void grid_fwd_kernel(const float *__restrict__ params,
                                                            GridOffs go, GridGeom g, int n_enc,
                                                            const int64_t *__restrict__ pairs,
                                                            const float *__restrict__ pos,
                                                            int64_t B, float *__restrict__ H0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * B * kL) return;
    const int64_t n = t / kL;
    const int l = (int)(t % kL);
    const int e = (n_enc == 2 && n >= B) ? 1 : 0;
    int idx[8];
    float w[8];
    row_corners(g, l, pairs, pos, B, n, idx, w);
    const f32x4 *grid = reinterpret_cast<const f32x4 *>(params + grid_off(go, e, l));
    f32x4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
#pragma unroll
    for (int cn = 0; cn < 8; ++cn) {
        const f32x4 c0 = grid[idx[cn] * 2], c1 = grid[idx[cn] * 2 + 1];
        a0 += w[cn] * c0;
        a1 += w[cn] * c1;
    }
    f32x4 *out = reinterpret_cast<f32x4 *>(H0 + n * kK0 + l * kF);
    out[0] = a0;
    out[1] = a1;
}

// ----------------------------------------------------------- grid bwd ----
// Scatter-add of dL/dh0 into the grid gradient: one wave per (row, level) item,
// lane = (corner c, feature f), so each atomic instruction of a wave updates the
// eight features of eight corner cells (eight 32-byte runs) instead of 64 scattered
// floats.  Every lane evaluates the trilinear lookup of the forward pass and keeps
// its own corner, so the weights are the forward's bit for bit.
__global__ __launch_bounds__(kThreads) void grid_bwd_kernel(float *__restrict__ grad, GridOffs go,
                                                            GridGeom g, int n_enc,
                                                            const int64_t *__restrict__ pairs,
                                                            const float *__restrict__ pos,
                                                            int64_t B, int64_t row0, int64_t rows,
                                                            const float *__restrict__ dH0) {
    const int lane = threadIdx.x & 63, c = lane >> 3, f = lane & 7;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t it = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); it < rows * kL;
         it += waves) {
        const int64_t n = row0 + it / kL;
        const int l = (int)(it % kL);
        const int e = (n_enc == 2 && n >= B) ? 1 : 0;
        int idx[8];
        float w[8];
        row_corners(g, l, pairs, pos, B, n, idx, w);
        int ic = idx[0];
        float wc = w[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            ic = c == k ? idx[k] : ic;
            wc = c == k ? w[k] : wc;
        }
        const float d = dH0[n * kK0 + l * kF + f];
        if (wc != 0.f) unsafeAtomicAdd(grad + grid_off(go, e, l) + (int64_t)ic * kF + f, wc * d);
    }
}

// ----------------------------------------------------- row-wise MFMA ----
enum { EPI_BIAS = 0, EPI_BIAS_RELU = 1, EPI_MASK = 2, EPI_PLAIN = 3 };

__device__ __forceinline__ bf16x8 load_row8(const float *__restrict__ X, int64_t rows, int64_t r,
                                            int ld, int k0) {
    bf16x8 b;
    if (r < rows) {
        const f32x4 *p = reinterpret_cast<const f32x4 *>(X + r * ld + k0);
        const f32x4 u = p[0], w = p[1];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            b[e] = f2bf(u[e]);
            b[4 + e] = f2bf(w[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) b[e] = f2bf(0.f);
    }
    return b;
}

// Y[rows][NOUT] = epi(X[rows][KIN] * A^T) with A[i][k] = W[i*w_si + k*w_sk].
template <int KIN, int NOUT, int EPI>
__global__ __launch_bounds__(kThreads) void rows_mma_kernel(
    const float *__restrict__ X, int64_t rows, const float *__restrict__ W, int w_si, int w_sk,
    const float *__restrict__ bias, const float *__restrict__ mask, float *__restrict__ Y) {
    constexpr int KB = KIN / 16, OB = NOUT / 32;
    __shared__ bf16x8 s_a[OB * KB * 64];
    __shared__ float s_bias[NOUT];
    __bf16 *sa = reinterpret_cast<__bf16 *>(s_a);
    for (int idx = threadIdx.x; idx < NOUT * KIN; idx += kThreads) {
        const int i = idx / KIN, k = idx % KIN;
        const float wv = W[(int64_t)i * w_si + (int64_t)k * w_sk];
        const int ob = i >> 5, il = i & 31, kb = k >> 4, hh = (k >> 3) & 1, e = k & 7;
        sa[((ob * KB + kb) * 64 + hh * 32 + il) * 8 + e] = f2bf(wv);
    }
    if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU)
        for (int i = threadIdx.x; i < NOUT; i += kThreads) s_bias[i] = bias[i];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, jl = lane & 31;
    const int64_t ntiles = ceil_div(rows, 64);
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles;
         tile += (int64_t)gridDim.x * 4) {
        f32x16 acc[OB][2];
#pragma unroll
        for (int ob = 0; ob < OB; ++ob)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[ob][0][r] = acc[ob][1][r] = 0.f;
        const int64_t r0 = tile * 64 + jl, r1 = r0 + 32;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const bf16x8 b0 = load_row8(X, rows, r0, KIN, kb * 16 + 8 * h);
            const bf16x8 b1 = load_row8(X, rows, r1, KIN, kb * 16 + 8 * h);
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) {
                const bf16x8 a = s_a[(ob * KB + kb) * 64 + lane];
                acc[ob][0] = mfma32(a, b0, acc[ob][0]);
                acc[ob][1] = mfma32(a, b1, acc[ob][1]);
            }
        }
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const int64_t row = tile * 64 + jb * 32 + jl;
            if (row >= rows) continue;
#pragma unroll
            for (int ob = 0; ob < OB; ++ob)
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    const int i0 = ob * 32 + 8 * gq + 4 * h;
                    f32x4 v;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = acc[ob][jb][4 * gq + e];
                    if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] += s_bias[i0 + e];
                    }
                    if (EPI == EPI_BIAS_RELU) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = v[e] > 0.f ? v[e] : 0.f;
                    }
                    if (EPI == EPI_MASK) {
                        const f32x4 m = *reinterpret_cast<const f32x4 *>(mask + row * NOUT + i0);
#pragma unroll
                        for (int e = 0; e < 4; ++e) v[e] = m[e] > 0.f ? v[e] : 0.f;
                    }
                    *reinterpret_cast<f32x4 *>(Y + row * NOUT + i0) = v;
                }
        }
    }
}

// ------------------------------------------------------- weight grads ----
constexpr int kLD = 64 + 8;  // bf16 per LDS row of a transposed 64-row tile

// dW[128][KIN] += sum_rows G[row][o] X[row][k];  db[o] += sum_rows G[row][o]
template <int KIN>
__global__ __launch_bounds__(kThreads) void wgrad_kernel(const float *__restrict__ G,
                                                         const float *__restrict__ X,
                                                         int64_t rows, float *__restrict__ dW,
                                                         float *__restrict__ db) {
    constexpr int JB = KIN / 32;
    __shared__ __attribute__((aligned(16))) __bf16 s_g[kH * kLD];
    __shared__ __attribute__((aligned(16))) __bf16 s_x[KIN * kLD];
    __shared__ float s_red[8][kH];
    const int tid = threadIdx.x;
    const int lane = tid & 63, ob = tid >> 6, h = lane >> 5, jl = lane & 31;
    f32x16 acc[JB];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[jb][r] = 0.f;
    float bsum[4] = {0.f, 0.f, 0.f, 0.f};
    const int c4 = tid & 31;
    const int64_t ntiles = ceil_div(rows, 64);
    // the next tile's rows are loaded into registers while the current one's
    // MFMAs run
    constexpr int XQ = 64 * KIN / 4;             // float4 per X tile
    constexpr int XPT = XQ / kThreads;           // per thread
    f32x4 gv[8], xv[XPT];
    auto fetch = [&](int64_t tile) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int64_t gr = tile * 64 + s * 8 + (tid >> 5);
            gv[s] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (gr < rows) gv[s] = *reinterpret_cast<const f32x4 *>(G + gr * kH + 4 * c4);
        }
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int q = tid + i * kThreads;
            const int64_t gr = tile * 64 + q / (KIN / 4);
            xv[i] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (gr < rows) xv[i] = *reinterpret_cast<const f32x4 *>(X + gr * KIN + 4 * (q % (KIN / 4)));
        }
    };
    if ((int64_t)blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int row = s * 8 + (tid >> 5);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bsum[e] += gv[s][e];
                s_g[(4 * c4 + e) * kLD + row] = f2bf(gv[s][e]);
            }
        }
#pragma unroll
        for (int i = 0; i < XPT; ++i) {
            const int q = tid + i * kThreads;
            const int row = q / (KIN / 4), cc = q % (KIN / 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) s_x[(4 * cc + e) * kLD + row] = f2bf(xv[i][e]);
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) fetch(tile + gridDim.x);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&s_g[(ob * 32 + jl) * kLD + kb * 16 + 8 * h]);
#pragma unroll
            for (int jb = 0; jb < JB; ++jb) {
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8 *>(&s_x[(jb * 32 + jl) * kLD + kb * 16 + 8 * h]);
                acc[jb] = mfma32(a, b, acc[jb]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = ob * 32 + d_row(r, lane);
            unsafeAtomicAdd(dW + o * KIN + jb * 32 + jl, acc[jb][r]);
        }
#pragma unroll
    for (int e = 0; e < 4; ++e) s_red[tid >> 5][4 * c4 + e] = bsum[e];
    __syncthreads();
    if (tid < kH) {
        float s = 0.f;
        for (int p = 0; p < 8; ++p) s += s_red[p][tid];
        unsafeAtomicAdd(db + tid, s);
    }
}

// ------------------------------------------------------- small kernels ----
// M[b] = E[b] * E[B + b] over latents of `width` features (128, or the 32 grid
// features of a grid-only network)
__global__ void merge_fwd_kernel(const float *__restrict__ E, int64_t B, float *__restrict__ M,
                                 int width) {
    const int64_t n4 = B * width / 4;
    const f32x4 *a = reinterpret_cast<const f32x4 *>(E);
    const f32x4 *b = reinterpret_cast<const f32x4 *>(E + B * width);
    f32x4 *m = reinterpret_cast<f32x4 *>(M);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        m[i] = a[i] * b[i];
}

__global__ void merge_bwd_kernel(const float *__restrict__ dM, const float *__restrict__ E,
                                 int64_t B, float *__restrict__ dE, int width) {
    const int64_t n4 = B * width / 4;
    const f32x4 *d = reinterpret_cast<const f32x4 *>(dM);
    const f32x4 *a = reinterpret_cast<const f32x4 *>(E);
    const f32x4 *b = reinterpret_cast<const f32x4 *>(E + B * width);
    f32x4 *da = reinterpret_cast<f32x4 *>(dE);
    f32x4 *dbp = reinterpret_cast<f32x4 *>(dE + B * width);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const f32x4 g = d[i];
        da[i] = g * b[i];
        dbp[i] = g * a[i];
    }
}

// y = w6 . d2 + b6; with targets: gy = sign(y - t) / B and per-block sums of |y - t|.
__global__ __launch_bounds__(kThreads) void head_fwd_kernel(
    const float *__restrict__ D2, const float *__restrict__ w6, const float *__restrict__ b6,
    const float *__restrict__ targets, int64_t B, float *__restrict__ y, float *__restrict__ gy,
    double *__restrict__ partial) {
    __shared__ float s_w[kH];
    __shared__ double s_sum[kThreads / 64];
    for (int i = threadIdx.x; i < kH; i += kThreads) s_w[i] = w6[i];
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double ab = 0.0;
    if (b < B) {
        const f32x4 *d = reinterpret_cast<const f32x4 *>(D2 + b * kH);
        float s = 0.f;
#pragma unroll 8
        for (int q = 0; q < kH / 4; ++q) {
            const f32x4 v = d[q];
            s = fmaf(v[0], s_w[4 * q], s);
            s = fmaf(v[1], s_w[4 * q + 1], s);
            s = fmaf(v[2], s_w[4 * q + 2], s);
            s = fmaf(v[3], s_w[4 * q + 3], s);
        }
        const float yy = s + b6[0];
        y[b] = yy;
        if (targets) {
            const float r = yy - targets[b];
            gy[b] = (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) / (float)B;
            ab = fabs((double)r);
        }
    }
    if (targets) {
        ab = wave_sum_f64(ab);
        if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = ab;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kThreads / 64; ++i) t += s_sum[i];
            partial[blockIdx.x] = t;
        }
    }
}

// Mean of the per-block sums; a non-finite loss (a NaN or infinite target or
// output) sets the call's status word, which stops the optimiser step.
__global__ void loss_reduce_kernel(const double *__restrict__ partial, int n, int64_t B,
                                   float *__restrict__ loss, int32_t *__restrict__ status) {
    __shared__ double s[64];
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) t += partial[i];
    s[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int i = 0; i < 64; ++i) a += s[i];
        const float l = (float)(a / (double)B);
        loss[0] = l;
        if (!isfinite(l)) status[0] = NDF_E_NONFINITE;
    }
}

// dPre5 = gy w6 (masked by d2 > 0);  gw6 += sum_b gy d2;  gb6 += sum_b gy
__global__ __launch_bounds__(kThreads) void head_bwd_kernel(const float *__restrict__ D2,
                                                            const float *__restrict__ gy,
                                                            const float *__restrict__ w6, int64_t B,
                                                            float *__restrict__ dpre,
                                                            float *__restrict__ gw6,
                                                            float *__restrict__ gb6) {
    __shared__ float s_red[2][kH];
    __shared__ float s_b[2];
    const int c = threadIdx.x & (kH - 1);
    const int ph = threadIdx.x >> 7;
    const float wc = w6[c];
    float acc = 0.f, accb = 0.f;
    for (int64_t b = (int64_t)blockIdx.x * 2 + ph; b < B; b += (int64_t)gridDim.x * 2) {
        const float g = gy[b];
        const float d = D2[b * kH + c];
        dpre[b * kH + c] = d > 0.f ? g * wc : 0.f;
        acc = fmaf(g, d, acc);
        accb += g;
    }
    s_red[ph][c] = acc;
    if (c == 0) s_b[ph] = accb;
    __syncthreads();
    if (threadIdx.x < kH) unsafeAtomicAdd(gw6 + c, s_red[0][c] + s_red[1][c]);
    if (threadIdx.x == 0) unsafeAtomicAdd(gb6, s_b[0] + s_b[1]);
}

__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float c1, float c2,
                            const int32_t *__restrict__ status) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    if (status[0] != NDF_OK) return;  // the step's loss was not finite: keep p, m, v
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// ------------------------------------------------------------ host side ----
namespace {

struct TrainWS {
    int32_t *status;
    float *H0, *H1, *H2, *E, *M, *D1, *D2, *y, *gy, *dA, *dB, *dH0;
    double *partial;
    size_t bytes;
};

TrainWS carve(void *ws, int64_t B) {
    TrainWS t{};
    const int64_t R = 2 * B;
    char *base = (char *)ws;
    size_t pos = 0;
    auto take = [&](size_t n) {
        char *p = base ? base + pos : nullptr;
        pos += align_up(n, 256);
        return p;
    };
    t.status = (int32_t *)take(kStatusBytes);
    t.H0 = (float *)take(R * kK0 * 4);
    t.H1 = (float *)take(R * kH * 4);
    t.H2 = (float *)take(R * kH * 4);
    t.E = (float *)take(R * kH * 4);
    t.M = (float *)take(B * kH * 4);
    t.D1 = (float *)take(B * kH * 4);
    t.D2 = (float *)take(B * kH * 4);
    t.y = (float *)take(B * 4);
    t.gy = (float *)take(B * 4);
    t.dA = (float *)take(R * kH * 4);
    t.dB = (float *)take(R * kH * 4);
    t.dH0 = (float *)take(R * kK0 * 4);
    t.partial = (double *)take(ceil_div(B, kThreads) * 8);
    t.bytes = pos;
    return t;
}

unsigned mma_blocks(int64_t rows) {
    int64_t b = ceil_div(ceil_div(rows, 64), 4);
    return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}
unsigned wgrad_blocks(int64_t rows) {
    int64_t b = ceil_div(rows, 64);
    return (unsigned)(b < 512 ? (b > 0 ? b : 1) : 512);  // 2 per CU: 222 -> 156 us at 2^19 rows
}

GridOffs grid_offs(const NetOffsets &o) {
    GridOffs g{};
    for (int e = 0; e < 2; ++e)
        for (int l = 0; l < kL; ++l) g.off[e][l] = o.grid[e][l];
    return g;
}

void encode_merge_layer4(const ndf_net_config *c, const NetOffsets &o, const float *P, int64_t B,
                         const TrainWS &t, hipStream_t st);

// Forward pass into the workspace; with targets also the loss and gy.
void forward(const ndf_net_config *c, const NetOffsets &o, const float *P, const int64_t *pairs,
             const float *pos, const float *targets, int64_t B, const TrainWS &t,
             hipStream_t st) {
    const int64_t R = 2 * B;
    const GridGeom g = grid_geom(c);
    const GridOffs go = grid_offs(o);
    hipLaunchKernelGGL(grid_fwd_kernel, dim3((unsigned)ceil_div(R * kL, kThreads)), dim3(kThreads),
                       0, st, P, go, g, c->n_enc, pairs, pos, B, t.H0);
    if (c->grid_only) {
        // the grid features are the latents: merge them and decode (W4 is [128][32])
        hipLaunchKernelGGL(merge_fwd_kernel, dim3(gs_blocks(B * kK0 / 4)), dim3(kThreads), 0, st,
                           t.H0, B, t.M, kK0);
        hipLaunchKernelGGL((rows_mma_kernel<kK0, kH, EPI_BIAS_RELU>), dim3(mma_blocks(B)),
                           dim3(kThreads), 0, st, t.M, B, P + o.W4, kK0, 1, P + o.b4, nullptr,
                           t.D1);
    } else {
        encode_merge_layer4(c, o, P, B, t, st);
    }
    hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_BIAS_RELU>), dim3(mma_blocks(B)),
                       dim3(kThreads), 0, st, t.D1, B, P + o.W5, kH, 1, P + o.b5, nullptr, t.D2);
    hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)ceil_div(B, kThreads)), dim3(kThreads), 0,
                       st, t.D2, P + o.w6, P + o.b6, targets, B, t.y, t.gy, t.partial);
}

// Encoder layers of both endpoints, the latent product and decoder layer 4.
void encode_merge_layer4(const ndf_net_config *c, const NetOffsets &o, const float *P, int64_t B,
                         const TrainWS &t, hipStream_t st) {
    const int64_t R = 2 * B;
    const int n_enc = c->n_enc;
    for (int e = 0; e < n_enc; ++e) {
        const int64_t r0 = n_enc == 1 ? 0 : e * B, rows = n_enc == 1 ? R : B;
        hipLaunchKernelGGL((rows_mma_kernel<kK0, kH, EPI_BIAS_RELU>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, t.H0 + r0 * kK0, rows, P + o.W1[e], kK0, 1,
                           P + o.b1[e], nullptr, t.H1 + r0 * kH);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_BIAS_RELU>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, t.H1 + r0 * kH, rows, P + o.W2[e], kH, 1,
                           P + o.b2[e], nullptr, t.H2 + r0 * kH);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_BIAS>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, t.H2 + r0 * kH, rows, P + o.W3[e], kH, 1,
                           P + o.b3[e], nullptr, t.E + r0 * kH);
    }
    hipLaunchKernelGGL(merge_fwd_kernel, dim3(gs_blocks(B * kH / 4)), dim3(kThreads), 0, st, t.E, B,
                       t.M, kH);
    hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_BIAS_RELU>), dim3(mma_blocks(B)),
                       dim3(kThreads), 0, st, t.M, B, P + o.W4, kH, 1, P + o.b4, nullptr, t.D1);
}

}  // namespace

size_t net_train_ws_bytes(const ndf_net_config *c, int64_t B) {
    (void)c;
    return carve(nullptr, B).bytes;
}

int launch_net_init(const ndf_net_config *c, float *params, float *opt, uint64_t seed,
                    hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    hipLaunchKernelGGL(fill_kernel, dim3(gs_blocks(o.total)), dim3(kThreads), 0, st, params,
                       o.total, 0.f);
    if (opt)
        hipLaunchKernelGGL(fill_kernel, dim3(gs_blocks(2 * o.total)), dim3(kThreads), 0, st, opt,
                           2 * o.total, 0.f);
    auto uni = [&](int64_t off, int64_t n, float a) {
        hipLaunchKernelGGL(uniform_kernel, dim3(gs_blocks(n)), dim3(kThreads), 0, st, params + off,
                           n, a, seed, off);
    };
    for (int e = 0; e < c->n_enc; ++e) {
        for (int l = 0; l < kL; ++l) uni(o.grid[e][l], o.cells[l] * kF, 1e-4f);
        if (c->grid_only) continue;
        uni(o.W1[e], kH * kK0, sqrtf(6.f / kK0));
        uni(o.W2[e], kH * kH, sqrtf(6.f / kH));
        uni(o.W3[e], kH * kH, sqrtf(6.f / kH));
    }
    const int k4 = c->grid_only ? kK0 : kH;  // inputs of the first decoder layer
    uni(o.W4, kH * k4, sqrtf(6.f / k4));
    uni(o.W5, kH * kH, sqrtf(6.f / kH));
    uni(o.w6, kH, sqrtf(6.f / kH));
    return status_of_launch();
}

int launch_net_forward(const ndf_net_config *c, const float *params, const int64_t *pairs,
                       const float *pos, int64_t B, float *y, void *ws, hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    TrainWS t = carve(ws, B);
    t.y = y;
    forward(c, o, params, pairs, pos, nullptr, B, t, st);
    return status_of_launch();
}

int launch_net_grad(const ndf_net_config *c, const float *P, const int64_t *pairs,
                    const float *pos, const float *targets, int64_t B, float *G, float *loss,
                    void *ws, hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    const TrainWS t = carve(ws, B);
    const int64_t R = 2 * B;
    launch_status_clear(t.status, st);
    hipLaunchKernelGGL(fill_kernel, dim3(gs_blocks(o.total)), dim3(kThreads), 0, st, G, o.total,
                       0.f);
    forward(c, o, P, pairs, pos, targets, B, t, st);
    const int nparts = (int)ceil_div(B, kThreads);
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(64), 0, st, t.partial, nparts, B, loss,
                       t.status);
    // decoder adjoint
    {
        int64_t hb = ceil_div(B, 2);
        hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)(hb < 1024 ? hb : 1024)), dim3(kThreads),
                           0, st, t.D2, t.gy, P + o.w6, B, t.dA, G + o.w6, G + o.b6);
    }
    hipLaunchKernelGGL(wgrad_kernel<kH>, dim3(wgrad_blocks(B)), dim3(kThreads), 0, st, t.dA, t.D1, B,
                       G + o.W5, G + o.b5);
    hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_MASK>), dim3(mma_blocks(B)), dim3(kThreads), 0,
                       st, t.dA, B, P + o.W5, 1, kH, nullptr, t.D1, t.dB);
    const GridGeom g = grid_geom(c);
    const GridOffs go = grid_offs(o);
    const int n_enc = c->n_enc;
    if (c->grid_only) {
        // W4 [128][32] on the merged grid features; the product rule gives the
        // grid features' gradient directly
        hipLaunchKernelGGL(wgrad_kernel<kK0>, dim3(wgrad_blocks(B)), dim3(kThreads), 0, st, t.dB,
                           t.M, B, G + o.W4, G + o.b4);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kK0, EPI_PLAIN>), dim3(mma_blocks(B)),
                           dim3(kThreads), 0, st, t.dB, B, P + o.W4, 1, kK0, nullptr, nullptr,
                           t.dA);
        hipLaunchKernelGGL(merge_bwd_kernel, dim3(gs_blocks(B * kK0 / 4)), dim3(kThreads), 0, st,
                           t.dA, t.H0, B, t.dH0, kK0);
        for (int e = 0; e < n_enc; ++e) {
            const int64_t r0 = n_enc == 1 ? 0 : e * B, rows = n_enc == 1 ? R : B;
            const int64_t items = rows * kL, per_block = kThreads / 64;
            const int64_t gb = ceil_div(items, per_block);
            hipLaunchKernelGGL(grid_bwd_kernel, dim3((unsigned)(gb < 16384 ? gb : 16384)),
                               dim3(kThreads), 0, st, G, go, g, n_enc, pairs, pos, B, r0, rows,
                               t.dH0);
        }
        return status_of_launch();
    }
    hipLaunchKernelGGL(wgrad_kernel<kH>, dim3(wgrad_blocks(B)), dim3(kThreads), 0, st, t.dB, t.M, B,
                       G + o.W4, G + o.b4);
    hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_PLAIN>), dim3(mma_blocks(B)), dim3(kThreads), 0,
                       st, t.dB, B, P + o.W4, 1, kH, nullptr, nullptr, t.dA);
    // product rule across the merge: dE[b] = dM[b] * E[B+b], dE[B+b] = dM[b] * E[b]
    hipLaunchKernelGGL(merge_bwd_kernel, dim3(gs_blocks(B * kH / 4)), dim3(kThreads), 0, st, t.dA,
                       t.E, B, t.dB, kH);
    // encoder adjoint(s): with a shared encoder both branches accumulate into one set
    for (int e = 0; e < n_enc; ++e) {
        const int64_t r0 = n_enc == 1 ? 0 : e * B, rows = n_enc == 1 ? R : B;
        float *dE = t.dB + r0 * kH, *dP2 = t.dA + r0 * kH, *dP1 = t.dB + r0 * kH;
        hipLaunchKernelGGL(wgrad_kernel<kH>, dim3(wgrad_blocks(rows)), dim3(kThreads), 0, st, dE,
                           t.H2 + r0 * kH, rows, G + o.W3[e], G + o.b3[e]);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_MASK>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, dE, rows, P + o.W3[e], 1, kH, nullptr,
                           t.H2 + r0 * kH, dP2);
        hipLaunchKernelGGL(wgrad_kernel<kH>, dim3(wgrad_blocks(rows)), dim3(kThreads), 0, st, dP2,
                           t.H1 + r0 * kH, rows, G + o.W2[e], G + o.b2[e]);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kH, EPI_MASK>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, dP2, rows, P + o.W2[e], 1, kH, nullptr,
                           t.H1 + r0 * kH, dP1);
        hipLaunchKernelGGL(wgrad_kernel<kK0>, dim3(wgrad_blocks(rows)), dim3(kThreads), 0, st, dP1,
                           t.H0 + r0 * kK0, rows, G + o.W1[e], G + o.b1[e]);
        hipLaunchKernelGGL((rows_mma_kernel<kH, kK0, EPI_PLAIN>), dim3(mma_blocks(rows)),
                           dim3(kThreads), 0, st, dP1, rows, P + o.W1[e], 1, kK0, nullptr, nullptr,
                           t.dH0 + r0 * kK0);
        const int64_t items = rows * kL, per_block = kThreads / 64;
        const int64_t gb = ceil_div(items, per_block);
        hipLaunchKernelGGL(grid_bwd_kernel, dim3((unsigned)(gb < 16384 ? gb : 16384)),
                           dim3(kThreads), 0, st, G, go, g, n_enc, pairs, pos, B, r0, rows,
                           t.dH0);
    }
    return status_of_launch();
}

int launch_adam(const ndf_net_config *c, float *params, float *opt, const float *grad,
                int64_t step, float lr, const int32_t *status, hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    const double c1 = 1.0 / (1.0 - pow(0.9, (double)step));
    const double c2 = 1.0 / (1.0 - pow(0.999, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3(gs_blocks(o.total)), dim3(kThreads), 0, st, params, opt,
                       opt + o.total, grad, o.total, lr, (float)c1, (float)c2, status);
    return status_of_launch();
}

// Phi_{nu mu} from Phi_{mu nu} (Sec. 6.4): the two encoder blocks [grid0..b3_0]
// and [grid1..b3_1] have the same layout and length, so out is in with the two
// ranges exchanged and the decoder copied.
__global__ void swap_encoders_kernel(const float *__restrict__ in, float *__restrict__ out,
                                     int64_t e0, int64_t e1, int64_t total) {
    const int64_t len = e1 - e0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kThreads) {
        int64_t src = i;
        if (i >= e0 && i < e1)
            src = i + len;
        else if (i >= e1 && i < e1 + len)
            src = i - len;
        out[i] = in[src];
    }
}

int launch_net_swap_encoders(const ndf_net_config *c, const float *in, float *out,
                             hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    // encoder 1 starts where encoder 0 ends; both end before W4
    const int64_t e0 = o.grid[0][0], e1 = o.grid[1][0];
    hipLaunchKernelGGL(swap_encoders_kernel, dim3(gs_blocks(o.total)), dim3(kThreads), 0, st, in,
                       out, e0, e1, o.total);
    return status_of_launch();
}

}  // namespace ndf
