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
// Scatter-add of dL/dh0 into the grid gradient: a wave takes four (row, level)
// items, lane = (item i, corner bit dx, feature f).  Each lane evaluates its
// item's trilinear lookup (the forward's arithmetic, so the same weights bit for
// bit) and issues one atomic per corner pair (dx = 0, 1 at equal dy, dz): on a
// dense level the two cells are neighbours in memory, so every atomic
// instruction of the wave adds four 64-byte runs.
__global__ __launch_bounds__(kThreads) void grid_bwd_kernel(float *__restrict__ grad, GridOffs go,
                                                            GridGeom g, int n_enc,
                                                            const int64_t *__restrict__ pairs,
                                                            const float *__restrict__ pos,
                                                            int64_t B, int64_t row0, int64_t rows,
                                                            const float *__restrict__ dH0) {
    const int lane = threadIdx.x & 63, i = lane >> 4, dx = (lane >> 3) & 1, f = lane & 7;
    const int64_t items = rows * kL;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t w0 = ((int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * 4;
         w0 < items; w0 += waves * 4) {
        const int64_t it = w0 + i;
        if (it >= items) continue;
        const int64_t n = row0 + it / kL;
        const int l = (int)(it % kL);
        const int e = (n_enc == 2 && n >= B) ? 1 : 0;
        int idx[8];
        float w[8];
        row_corners(g, l, pairs, pos, B, n, idx, w);
        const float d = dH0[n * kK0 + l * kF + f];
        float *gl = grad + grid_off(go, e, l) + f;
        // this lane's corner of each pair by bit blending (a select between two
        // elements is turned into a lane-dependent index, which moves idx and w
        // to memory)
        const int m = -dx;
        int ic[4];
        float wc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ic[c] = idx[2 * c] ^ (m & (idx[2 * c] ^ idx[2 * c + 1]));
            wc[c] = __int_as_float(__float_as_int(w[2 * c]) ^
                                   (m & (__float_as_int(w[2 * c]) ^ __float_as_int(w[2 * c + 1]))));
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (wc[c] != 0.f) unsafeAtomicAdd(gl + (int64_t)ic[c] * kF, wc[c] * d);
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
                bsum[e] += (float)f2bf(gv[s][e]);  // the bf16 G that the MFMA takes
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
        acc = fmaf(g, (float)f2bf(d), acc);  // d2 as a bf16 operand, like every weight grad
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
int64_t grid_bwd_blocks(int64_t rows) {
    const int64_t b = ceil_div(rows * kL, 4 * (kThreads / 64));  // 4 items per wave
    return b < 8192 ? (b > 0 ? b : 1) : 8192;
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

// ========================================================== fused step ====
// The step of a network with one encoder shared by both endpoints (the
// symmetric pair encoding of Sec. 4.1) runs in four kernels: a forward kernel
// (grid gather, encoder for both endpoints, latent product, decoder, head, the
// L1 loss and its gradient), a backward kernel (the data adjoint from the head
// back to dL/dh0), the grid scatter (grid_bwd_kernel) and one kernel for every
// weight and bias gradient.  A wave takes 32 pairs: the first endpoints are
// MFMA column block q = 0, the second endpoints q = 1, so both share every
// weight fragment and the latent product is register-local; the decoder runs
// on the pair rows (q = 0).
// What the backward pass and the weight gradients need is stored per 32-row
// block ("slab") in the register order of the MFMA operands: chunk (kb, lane)
// = 16 bytes = row lane % 32, features feat_perm(kb, lane / 32, e) for layer
// outputs (the order the MFMA accumulators pack into) and feat_nat for the grid
// features h0.  Every store and load of a slab is a coalesced 16-byte access.
// Numerics are those of the layer-by-layer kernels: bf16 operands into every
// MFMA, FP32 accumulators, FP32 latents into the product; the stored operands
// of the weight gradients are the same bf16 values the MFMAs take, and bias
// gradients sum those bf16 values (a bias is the weight of a constant input 1).
__host__ __device__ inline int feat_perm(int kb, int h, int e) {
    return 16 * kb + 8 * (e >> 2) + 4 * h + (e & 3);
}
__host__ __device__ inline int feat_nat(int kb, int h, int e) { return 16 * kb + 8 * h + e; }

constexpr int kTW = 8;                 // waves per workgroup of the fused kernels
constexpr int kTThreads = 64 * kTW;
constexpr int kFragH = 4 * 8 * 64;     // bf16x8 per 128 x 128 layer fragment set
constexpr int kFrag1 = 4 * 2 * 64;     // W1 (128 x 32), and W1^T (32 x 128): 8 x 64
constexpr int kFrag1F = 4 * 7 * 64;    // W1 with Fourier features (128 x 112)

// Packed weights of one step: forward A fragments of W1..W5 (W[o][k], lane l
// of fragment (ob, kb) holds row 32 ob + l % 32, inputs 8 (l / 32) + 16 kb + e in
// the order of the layer's input), then the adjoint's A fragments of
// W1^T..W5^T (row = the layer's input k, inputs = its outputs o in the packed
// gradient's order feat_perm).
struct TrainFrags {
    bf16x8 *f[5];
    bf16x8 *t[5];
};

__global__ void pack_train_kernel(const float *__restrict__ P, int64_t w1, int64_t w2,
                                  int64_t w3, int64_t w4, int64_t w5, int kin1, TrainFrags F) {
    const int64_t wo[5] = {w1, w2, w3, w4, w5};
    // forward: W1 (128 x kin1) and W2..W5; adjoint: W1^T (the 32 grid inputs only:
    // no gradient flows into the Fourier features) and W2^T..W5^T
    const int n1 = kH * kin1, nf = n1 + 4 * kH * kH, na = kH * kK0 + 4 * kH * kH;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nf + na; t += gridDim.x * blockDim.x) {
        const bool adj = t >= nf;
        int u = adj ? t - nf : t;
        const int m1 = adj ? kH * kK0 : n1;
        const int L = u < m1 ? 0 : 1 + (u - m1) / (kH * kH);
        if (L > 0) u = (u - m1) % (kH * kH);
        const int KIN = L == 0 ? kin1 : kH;
        const int e = u & 7, lane = (u >> 3) & 63, fi = u >> 9;
        const int h = lane >> 5, il = lane & 31;
        float v;
        if (!adj) {
            const int KB = KIN / 16, ob = fi / KB, kb = fi % KB;
            const int k = L == 0 ? feat_nat(kb, h, e) : feat_perm(kb, h, e);
            v = P[wo[L] + (int64_t)(32 * ob + il) * KIN + k];
        } else {
            const int mb = fi / 8, kb = fi % 8;
            v = P[wo[L] + (int64_t)feat_perm(kb, h, e) * KIN + 32 * mb + il];
        }
        __bf16 *dst = reinterpret_cast<__bf16 *>(adj ? F.t[L] : F.f[L]);
        dst[u] = f2bf(v);
    }
}

struct FusedArgs {
    const float *P;
    int64_t grid[kL];  // offsets of the (single) encoder's grid levels in P
    const bf16x8 *wf[5], *wt[5];
    const float *b[5], *w6, *b6;
    GridGeom g;
    const int64_t *pairs;
    const float *pos;
    const float *targets;
    int64_t B;
    float inv_b;
    // slabs: enc = [2 T] (block 2 t + q), dec = [T]
    u32x4 *h0, *h1, *h2, *m, *d1, *d2, *da5, *da4, *dlat, *da2, *da1;
    f32x4 *lat;     // FP32 latents [2 T][4 ob][4 g][64]
    float *gy;      // [T * 32]
    float *y;       // [B] or null
    float *dh0;     // [2 B][32] FP32, rows q B + pair
    double *partial;
};

__device__ __forceinline__ int64_t slab_chunk(int64_t blk, int nkb, int kb, int lane) {
    return (blk * nkb + kb) * 64 + lane;
}

// Pack one output block's accumulators (acc index 8 s + e <-> chunk 2 ob + s,
// element e) into two bf16 chunks.
__device__ __forceinline__ void pack_block(const f32x16 &acc, u32x4 &c0, u32x4 &c1) {
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
        c0[e2] = pack_bf16x2(acc[2 * e2], acc[2 * e2 + 1]);
        c1[e2] = pack_bf16x2(acc[8 + 2 * e2], acc[8 + 2 * e2 + 1]);
    }
}

// Keep the halves of g whose forward activation (bf16 pair h, a ReLU output, so
// +0 or positive) is non-zero: the ReLU derivative on packed pairs.
__device__ __forceinline__ uint32_t relu_mask2(uint32_t g, uint32_t h) {
    const uint32_t lo = (h & 0xffffu) ? 0xffffu : 0u;
    const uint32_t hi = (h >> 16) ? 0xffff0000u : 0u;
    return g & (lo | hi);
}

// acc[q] = bias (or 0) + W-block ob x in[.][q] over KB k-blocks.
template <int KB, int NQ>
__device__ __forceinline__ void mma_block(const bf16x8 *__restrict__ wf, int ob,
                                          const float *__restrict__ bias_h,
                                          const bf16x8 (&in)[8][2], f32x16 (&acc)[2], int lane) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        f32x4 bv = {0.f, 0.f, 0.f, 0.f};
        if (bias_h) bv = *reinterpret_cast<const f32x4 *>(bias_h + 32 * ob + 8 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q][4 * g + i] = bv[i];
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const bf16x8 a = wf[(ob * KB + kb) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = mfma32(a, in[kb][q], acc[q]);
    }
}

// Grid features of one endpoint for k-block kb: lane half h gathers level
// 2 kb + h (8 FP32 features per cell, trilinear over 8 corners).
template <bool POS>
__device__ __forceinline__ bf16x8 gather_h0(const FusedArgs &A, int kb, int h, int64_t v,
                                            const float (&p)[3]) {
    const int l = 2 * kb + h;
    int R[3];
    level_dims(A.g, l, R);
    const uint32_t hm = level_hmask(A.g, l);
    int idx[8];
    float w[8];
    if (POS)
        corners_pos32<true>(R, p, idx, w, hm);
    else
        corners_R32<true>(A.g, R, v, idx, w, hm);
    const f32x4 *grid = reinterpret_cast<const f32x4 *>(A.P + (h ? A.grid[2 * kb + 1] : A.grid[2 * kb]));
    f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = s0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        // a corner of weight 0 adds nothing: on a level of the vertex grid's size
        // only one corner of eight has weight, so most lanes skip the other reads
        if (w[c] == 0.f) continue;
        const f32x4 c0 = grid[(int64_t)idx[c] * 2], c1 = grid[(int64_t)idx[c] * 2 + 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            s0[i] = fmaf(w[c], c0[i], s0[i]);
            s1[i] = fmaf(w[c], c1[i], s1[i]);
        }
    }
    bf16x8 t;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        t[i] = f2bf(s0[i]);
        t[4 + i] = f2bf(s1[i]);
    }
    return t;
}

__device__ __forceinline__ u32x4 as_u(const bf16x8 &v) { return __builtin_bit_cast(u32x4, v); }
__device__ __forceinline__ bf16x8 as_b(const u32x4 &v) { return __builtin_bit_cast(bf16x8, v); }

// Forward of 32 pairs per wave; with targets also the loss partial sums, gy and
// the first gradient da5 = gy w6 (masked by d2 > 0).
template <bool POS, bool FF>
__global__ __launch_bounds__(kTThreads) void train_fwd_kernel(FusedArgs A) {
    constexpr int KB1 = FF ? kK0F / 16 : kK0 / 16;  // k-blocks of the encoder input
    __shared__ bf16x8 s_w1[4 * KB1 * 64];
    __shared__ bf16x8 s_w[4][kFragH];
    __shared__ __attribute__((aligned(16))) float s_b[5][kH];
    __shared__ __attribute__((aligned(16))) float s_w6[kH];
    __shared__ double s_part[kTW];
    const int tid = threadIdx.x;
    for (int i = tid; i < 4 * KB1 * 64; i += kTThreads) s_w1[i] = A.wf[0][i];
    for (int L = 0; L < 4; ++L)
        for (int i = tid; i < kFragH; i += kTThreads) s_w[L][i] = A.wf[L + 1][i];
    for (int i = tid; i < 5 * kH; i += kTThreads) s_b[i / kH][i % kH] = A.b[i / kH][i % kH];
    for (int i = tid; i < kH; i += kTThreads) s_w6[i] = A.w6[i];
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, jl = lane & 31;
    const int64_t T = ceil_div(A.B, 32);
    const int64_t V = (int64_t)A.g.nx * A.g.ny * A.g.nz;
    const float b6 = A.b6[0];
    const float inv_b = 1.f / (float)A.B;
    double loss_part = 0.0;
    for (int64_t tile = (int64_t)blockIdx.x * kTW + wave; tile < T;
         tile += (int64_t)gridDim.x * kTW) {
        int h4 = 4 * h;
        asm volatile("" : "+v"(h4));
        const int64_t pair = tile * 32 + jl;
        const bool ok = pair < A.B;
        bf16x8 a[8][2], b[8][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int64_t v = 0;
            float p[3] = {0.f, 0.f, 0.f};
            if (ok) {
                if (POS) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) p[c] = A.pos[(2 * pair + q) * 3 + c];
                } else {
                    v = A.pairs[2 * pair + q];
                    v = v < 0 ? 0 : (v >= V ? V - 1 : v);  // out-of-range pairs are clamped
                }
            }
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                a[kb][q] = gather_h0<POS>(A, kb, h, v, p);
                A.h0[slab_chunk(2 * tile + q, KB1, kb, lane)] = as_u(a[kb][q]);
            }
            if (FF) {  // the raw position and its Fourier features
                float pp[3];
                if (POS)
                    clamp_p(p, pp);
                else
                    vertex_p(A.g, v, pp);
#pragma unroll
                for (int kb = 2; kb < KB1; ++kb) {
                    a[kb][q] = ff_chunk(kb, h, pp);
                    A.h0[slab_chunk(2 * tile + q, KB1, kb, lane)] = as_u(a[kb][q]);
                }
            }
        }
        f32x16 acc[2];
        // layer 1: 32 -> 128, ReLU (both endpoints)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<KB1, 2>(s_w1, ob, s_b[0] + h4, a, acc, lane);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                u32x4 c0, c1;
                pack_block(acc[q], c0, c1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    c0[i] = relu_bf16x2(c0[i]);
                    c1[i] = relu_bf16x2(c1[i]);
                }
                b[2 * ob][q] = as_b(c0);
                b[2 * ob + 1][q] = as_b(c1);
                A.h1[slab_chunk(2 * tile + q, 8, 2 * ob, lane)] = c0;
                A.h1[slab_chunk(2 * tile + q, 8, 2 * ob + 1, lane)] = c1;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 2: ReLU
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 2>(s_w[0], ob, s_b[1] + h4, b, acc, lane);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                u32x4 c0, c1;
                pack_block(acc[q], c0, c1);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    c0[i] = relu_bf16x2(c0[i]);
                    c1[i] = relu_bf16x2(c1[i]);
                }
                a[2 * ob][q] = as_b(c0);
                a[2 * ob + 1][q] = as_b(c1);
                A.h2[slab_chunk(2 * tile + q, 8, 2 * ob, lane)] = c0;
                A.h2[slab_chunk(2 * tile + q, 8, 2 * ob + 1, lane)] = c1;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 3: the latents (FP32, kept for the product rule) and their product
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 2>(s_w[1], ob, s_b[2] + h4, a, acc, lane);
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    f32x4 t;
#pragma unroll
                    for (int i = 0; i < 4; ++i) t[i] = acc[q][4 * g + i];
                    A.lat[((2 * tile + q) * 4 + ob) * 256 + g * 64 + lane] = t;
                }
            f32x16 mm;
#pragma unroll
            for (int r = 0; r < 16; ++r) mm[r] = acc[0][r] * acc[1][r];
            u32x4 c0, c1;
            pack_block(mm, c0, c1);
            b[2 * ob][0] = as_b(c0);
            b[2 * ob + 1][0] = as_b(c1);
            A.m[slab_chunk(tile, 8, 2 * ob, lane)] = c0;
            A.m[slab_chunk(tile, 8, 2 * ob + 1, lane)] = c1;
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 4: ReLU (pair rows)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 1>(s_w[2], ob, s_b[3] + h4, b, acc, lane);
            u32x4 c0, c1;
            pack_block(acc[0], c0, c1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c0[i] = relu_bf16x2(c0[i]);
                c1[i] = relu_bf16x2(c1[i]);
            }
            a[2 * ob][0] = as_b(c0);
            a[2 * ob + 1][0] = as_b(c1);
            A.d1[slab_chunk(tile, 8, 2 * ob, lane)] = c0;
            A.d1[slab_chunk(tile, 8, 2 * ob + 1, lane)] = c1;
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 5: ReLU, and the head y = w6 . d2 + b6 in FP32
        float part = 0.f;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 1>(s_w[3], ob, s_b[4] + h4, a, acc, lane);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4 wv = *reinterpret_cast<const f32x4 *>(s_w6 + h4 + 32 * ob + 8 * g);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[0][4 * g + i] = relu_f32(acc[0][4 * g + i]);
                    part = fmaf(wv[i], acc[0][4 * g + i], part);
                }
            }
            u32x4 c0, c1;
            pack_block(acc[0], c0, c1);
            b[2 * ob][0] = as_b(c0);
            b[2 * ob + 1][0] = as_b(c1);
            A.d2[slab_chunk(tile, 8, 2 * ob, lane)] = c0;
            A.d2[slab_chunk(tile, 8, 2 * ob + 1, lane)] = c1;
            __builtin_amdgcn_sched_barrier(0);
        }
        const float y = part + __shfl_xor(part, 32, 64) + b6;
        if (A.y && h == 0 && ok) A.y[pair] = y;
        if (A.targets) {
            const float r = ok ? y - A.targets[pair] : 0.f;
            const float gyv = (r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f)) * inv_b;
            if (h == 0) {
                A.gy[tile * 32 + jl] = gyv;
                loss_part += ok ? fabs((double)r) : 0.0;
            }
            // da5 = gy w6 where d2 > 0, in the packed order of d2
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const u32x4 dd = as_u(b[j][0]);
                u32x4 c;
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) {
                    const int f0 = feat_perm(j, 0, 2 * e2) + h4;
                    c[e2] = relu_mask2(pack_bf16x2(gyv * s_w6[f0], gyv * s_w6[f0 + 1]), dd[e2]);
                }
                A.da5[slab_chunk(tile, 8, j, lane)] = c;
            }
        }
    }
    if (A.targets) {
        loss_part = wave_sum_f64(loss_part);
        if (lane == 0) s_part[wave] = loss_part;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kTW; ++w) t += s_part[w];
            A.partial[blockIdx.x] = t;
        }
    }
}

// One encoder adjoint layer for both endpoints: out = pack(W^T in) masked by the
// forward activation hm > 0; the result is also stored as the layer's G slab.
__device__ __forceinline__ void adj_masked_layer(const bf16x8 *__restrict__ wt,
                                                 const u32x4 *__restrict__ hm,
                                                 u32x4 *__restrict__ gout, int64_t tile,
                                                 const bf16x8 (&in)[8][2], bf16x8 (&out)[8][2],
                                                 int lane) {
    f32x16 acc[2];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        mma_block<8, 2>(wt, ob, nullptr, in, acc, lane);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            u32x4 c0, c1;
            pack_block(acc[q], c0, c1);
            const u32x4 m0 = hm[slab_chunk(2 * tile + q, 8, 2 * ob, lane)];
            const u32x4 m1 = hm[slab_chunk(2 * tile + q, 8, 2 * ob + 1, lane)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c0[i] = relu_mask2(c0[i], m0[i]);
                c1[i] = relu_mask2(c1[i], m1[i]);
            }
            out[2 * ob][q] = as_b(c0);
            out[2 * ob + 1][q] = as_b(c1);
            gout[slab_chunk(2 * tile + q, 8, 2 * ob, lane)] = c0;
            gout[slab_chunk(2 * tile + q, 8, 2 * ob + 1, lane)] = c1;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Data adjoint of 32 pairs per wave: da5 -> da4 -> dlat (both endpoints) -> da2
// -> da1 -> dL/dh0 (FP32, rows q B + pair, for the grid scatter).  Every G slab
// is stored for the weight gradients.
__global__ __launch_bounds__(kTThreads) void train_bwd_kernel(FusedArgs A) {
    __shared__ bf16x8 s_t1[kFrag1];
    __shared__ bf16x8 s_t[4][kFragH];  // W2^T .. W5^T
    const int tid = threadIdx.x;
    for (int i = tid; i < kFrag1; i += kTThreads) s_t1[i] = A.wt[0][i];
    for (int L = 0; L < 4; ++L)
        for (int i = tid; i < kFragH; i += kTThreads) s_t[L][i] = A.wt[L + 1][i];
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, jl = lane & 31;
    const int64_t T = ceil_div(A.B, 32);
    for (int64_t tile = (int64_t)blockIdx.x * kTW + wave; tile < T;
         tile += (int64_t)gridDim.x * kTW) {
        const int64_t pair = tile * 32 + jl;
        const bool ok = pair < A.B;
        bf16x8 x[8][2], y[8][2];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) x[kb][0] = as_b(A.da5[slab_chunk(tile, 8, kb, lane)]);
        f32x16 acc[2];
        // W5^T: d(d1), masked by d1 > 0 -> da4
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 1>(s_t[3], ob, nullptr, x, acc, lane);
            u32x4 c0, c1;
            pack_block(acc[0], c0, c1);
            const u32x4 m0 = A.d1[slab_chunk(tile, 8, 2 * ob, lane)];
            const u32x4 m1 = A.d1[slab_chunk(tile, 8, 2 * ob + 1, lane)];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c0[i] = relu_mask2(c0[i], m0[i]);
                c1[i] = relu_mask2(c1[i], m1[i]);
            }
            y[2 * ob][0] = as_b(c0);
            y[2 * ob + 1][0] = as_b(c1);
            A.da4[slab_chunk(tile, 8, 2 * ob, lane)] = c0;
            A.da4[slab_chunk(tile, 8, 2 * ob + 1, lane)] = c1;
            __builtin_amdgcn_sched_barrier(0);
        }
        // W4^T: dm, then the product rule: dlat_A = dm lat_B, dlat_B = dm lat_A
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            mma_block<8, 1>(s_t[2], ob, nullptr, y, acc, lane);
            f32x16 la, lb;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4 ta = A.lat[((2 * tile) * 4 + ob) * 256 + g * 64 + lane];
                const f32x4 tb = A.lat[((2 * tile + 1) * 4 + ob) * 256 + g * 64 + lane];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    la[4 * g + i] = acc[0][4 * g + i] * tb[i];
                    lb[4 * g + i] = acc[0][4 * g + i] * ta[i];
                }
            }
            u32x4 c0, c1;
            pack_block(la, c0, c1);
            x[2 * ob][0] = as_b(c0);
            x[2 * ob + 1][0] = as_b(c1);
            A.dlat[slab_chunk(2 * tile, 8, 2 * ob, lane)] = c0;
            A.dlat[slab_chunk(2 * tile, 8, 2 * ob + 1, lane)] = c1;
            pack_block(lb, c0, c1);
            x[2 * ob][1] = as_b(c0);
            x[2 * ob + 1][1] = as_b(c1);
            A.dlat[slab_chunk(2 * tile + 1, 8, 2 * ob, lane)] = c0;
            A.dlat[slab_chunk(2 * tile + 1, 8, 2 * ob + 1, lane)] = c1;
            __builtin_amdgcn_sched_barrier(0);
        }
        // W3^T: dh2, masked by h2 > 0 -> da2;  W2^T: dh1, masked by h1 > 0 -> da1
        adj_masked_layer(s_t[1], A.h2, A.da2, tile, x, y, lane);
        adj_masked_layer(s_t[0], A.h1, A.da1, tile, y, x, lane);
        // W1^T: dL/dh0 (32 features: level g = 0..3, features 4 h + i)
        mma_block<8, 2>(s_t1, 0, nullptr, x, acc, lane);
        if (ok) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                float *dst = A.dh0 + ((int64_t)q * A.B + pair) * kK0 + 4 * h;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    f32x4 t;
#pragma unroll
                    for (int i = 0; i < 4; ++i) t[i] = acc[q][4 * g + i];
                    *reinterpret_cast<f32x4 *>(dst + 8 * g) = t;
                }
            }
        }
    }
}

// Weight and bias gradients of every layer in one launch: workgroup ranges
// [wg0[L], wg0[L + 1]) take layer L (0..4 = W1..W5, 5 = the head w6, b6), each
// workgroup a strided share of its layer's 64-row slab pairs.  A slab pair of
// G (the layer's output gradient) and X (its input) is loaded with 16-byte
// reads (4 rows x 8 features per thread), transposed in registers and written
// to LDS feature-major, s[f][row]; the waves then accumulate
// dW[o][k] += sum_rows G[row][o] X[row][k] on MFMA (K = rows) and threads
// f < 128 sum the bf16 G column f for the bias.  One atomic flush per workgroup
// at the end.
struct WgradArgs {
    const u32x4 *g[5], *x[5];
    int kin1;  // inputs of W1 (32, or 112 with Fourier features)
    int64_t nslab[6];
    float *dW[6], *db[6];
    const u32x4 *d2;
    const float *gy;
    int wg0[7];
};

constexpr int kWgLD = 64 + 8;  // bf16 per LDS feature row (64 rows + pad)

// rows r = 0..3 of 8 features each (c[r]) -> features e = 0..7 of 4 rows each
__device__ __forceinline__ void transpose4(const u32x4 (&c)[4], uint2 (&t)[8]) {
#pragma unroll
    for (int p = 0; p < 4; ++p)      // word p = features 2 p, 2 p + 1
#pragma unroll
        for (int i = 0; i < 2; ++i) {  // rows 2 i, 2 i + 1
            const uint32_t a = c[2 * i][p], b = c[2 * i + 1][p];
            const uint32_t lo = __builtin_amdgcn_perm(b, a, 0x05040100u);
            const uint32_t hi = __builtin_amdgcn_perm(b, a, 0x07060302u);
            if (i == 0) {
                t[2 * p].x = lo;
                t[2 * p + 1].x = hi;
            } else {
                t[2 * p].y = lo;
                t[2 * p + 1].y = hi;
            }
        }
}

// The 4 x 8 block (slab blk, k-block kb, half h, rows r0 .. r0 + 3) of a slab
// with nkb k-blocks: 4 coalesced 16-byte loads (zeros past the last slab) ...
__device__ __forceinline__ void load4(const u32x4 *__restrict__ src, int64_t blk, int64_t nslab,
                                      int nkb, int kb, int h, int r0, u32x4 (&c)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
        c[r] = blk < nslab ? src[slab_chunk(blk, nkb, kb, 32 * h + r0 + r)]
                           : u32x4{0u, 0u, 0u, 0u};
}
// ... written feature-major into s (the slab's rows at 32 sl).
__device__ __forceinline__ void write4(const u32x4 (&c)[4], int kb, int h, int r0, int sl,
                                       bool nat, __bf16 *__restrict__ s) {
    uint2 t[8];
    transpose4(c, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int f = nat ? feat_nat(kb, h, e) : feat_perm(kb, h, e);
        *reinterpret_cast<uint2 *>(s + f * kWgLD + 32 * sl + r0) = t[e];
    }
}

// Eight waves: wave w accumulates output rows 32 (w % 4) .. + 31 against input
// columns 64 (w / 4) .. + 63 (two 32-column blocks).  Threads t < 256 stage G
// (the head: t < 64 stage gy), t >= 256 stage X, four rows of one 8-feature
// block each; the next slab pair's loads are in flight while the MFMAs run.
__global__ __launch_bounds__(512) void wgrad_all_kernel(WgradArgs A) {
    __shared__ __attribute__((aligned(16))) __bf16 s_g[kH * kWgLD];
    __shared__ __attribute__((aligned(16))) __bf16 s_x[kH * kWgLD];
    __shared__ float s_gy[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, jl = lane & 31;
    int L = 0;
    while (L < 5 && (int)blockIdx.x >= A.wg0[L + 1]) ++L;
    const int part = (int)blockIdx.x - A.wg0[L], nparts = A.wg0[L + 1] - A.wg0[L];
    const int64_t nslab = A.nslab[L];
    if (2 * (int64_t)part >= nslab) return;
    const int kin = L == 0 ? A.kin1 : kH;
    const int xkb = kin / 16, xcb = (kin + 31) / 32;
    const int ob = wave & 3, cb0 = 2 * (wave >> 2);
    // this thread's block
    const int u = tid & 255, sl = u >> 7, kb = (u >> 4) & 7, hh = (u >> 3) & 1,
              r0 = 4 * (u & 7);
    const bool is_g = tid < 256;
    const bool active = L == 5 ? (is_g ? tid < 64 : true) : (is_g || kb < xkb);
    const u32x4 *src = L == 5 ? A.d2 : (is_g ? A.g[L] : A.x[L]);
    const int nkb = is_g ? 8 : xkb;
    const bool nat = !is_g && L == 0;
    u32x4 c[4];
    float gyv = 0.f;
    auto fetch = [&](int64_t sp) {
        if (!active) return;
        if (L == 5 && is_g) {
            const int64_t r = 2 * sp * 32 + tid;
            gyv = r < nslab * 32 ? A.gy[r] : 0.f;
        } else {
            load4(src, 2 * sp + sl, nslab, nkb, kb, hh, r0, c);
        }
    };
    f32x16 acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[q][r] = 0.f;
    float bsum = 0.f;
    fetch(part);
    for (int64_t sp = part; 2 * sp < nslab; sp += nparts) {
        if (active) {
            if (L == 5 && is_g)
                s_gy[tid] = gyv;
            else
                write4(c, kb, hh, r0, sl, nat, is_g && L != 5 ? s_g : s_x);
        }
        __syncthreads();
        if (2 * (sp + nparts) < nslab) fetch(sp + nparts);
        if (L == 5) {
            // dw6[k] = sum_rows gy d2[row][k] (thread k), db6 = sum_rows gy (thread 128)
            if (tid < kH) {
                const __bf16 *xr = s_x + tid * kWgLD;
#pragma unroll 8
                for (int r = 0; r < 64; ++r) bsum = fmaf(s_gy[r], (float)xr[r], bsum);
            } else if (tid == kH) {
                for (int r = 0; r < 64; ++r) bsum += s_gy[r];
            }
        } else {
            if (cb0 < xcb) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
                        s_g + (32 * ob + jl) * kWgLD + 16 * kk + 8 * h);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (cb0 + q >= xcb) continue;
                        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
                            s_x + (32 * (cb0 + q) + jl) * kWgLD + 16 * kk + 8 * h);
                        acc[q] = mfma32(a, b, acc[q]);
                    }
                }
            }
            if (tid < kH) {
                const u32x4 *gr = reinterpret_cast<const u32x4 *>(s_g + tid * kWgLD);
#pragma unroll
                for (int cc = 0; cc < 8; ++cc) {
                    const u32x4 v = gr[cc];
#pragma unroll
                    for (int i = 0; i < 4; ++i) bsum += bf_lo(v[i]) + bf_hi(v[i]);
                }
            }
        }
        __syncthreads();
    }
    if (L == 5) {
        if (tid < kH) unsafeAtomicAdd(A.dW[5] + tid, bsum);
        else if (tid == kH) unsafeAtomicAdd(A.db[5], bsum);
        return;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        // columns past the input width (W1 with 112 inputs: 112..127) hold
        // nothing and are not written
        if (cb0 + q >= xcb || 32 * (cb0 + q) + jl >= kin) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            unsafeAtomicAdd(A.dW[L] + (32 * ob + d_row(r, lane)) * kin + 32 * (cb0 + q) + jl,
                            acc[q][r]);
    }
    if (tid < kH) unsafeAtomicAdd(A.db[L] + tid, bsum);
}

// ------------------------------------------------------- fused host ----
static bool fused_path(const ndf_net_config *c) { return c->n_enc == 1 && !c->grid_only; }

struct FusedWS {
    int32_t *status;
    TrainFrags fr;
    u32x4 *h0, *h1, *h2, *m, *d1, *d2, *da5, *da4, *dlat, *da2, *da1;
    f32x4 *lat;
    float *gy, *dh0;
    double *partial;
    size_t bytes;
};

constexpr int kFusedBlocksMax = 512;

static FusedWS carve_fused(const ndf_net_config *c, void *ws, int64_t B) {
    FusedWS t{};
    const int64_t T = ceil_div(B, 32);
    char *base = (char *)ws;
    size_t pos = 0;
    auto take = [&](size_t n) {
        char *p = base ? base + pos : nullptr;
        pos += align_up(n, 256);
        return p;
    };
    t.status = (int32_t *)take(kStatusBytes);
    const int kb1 = enc_in(c) / 16;
    for (int L = 0; L < 5; ++L) t.fr.f[L] = (bf16x8 *)take((L == 0 ? 4 * kb1 * 64 : kFragH) * 16);
    for (int L = 0; L < 5; ++L) t.fr.t[L] = (bf16x8 *)take((L == 0 ? kFrag1 : kFragH) * 16);
    const size_t slab = 8 * 64 * 16;  // 128 features x 32 rows, bf16
    t.h0 = (u32x4 *)take(2 * T * kb1 * 64 * 16);
    t.h1 = (u32x4 *)take(2 * T * slab);
    t.h2 = (u32x4 *)take(2 * T * slab);
    t.lat = (f32x4 *)take(2 * T * 2 * slab);
    t.m = (u32x4 *)take(T * slab);
    t.d1 = (u32x4 *)take(T * slab);
    t.d2 = (u32x4 *)take(T * slab);
    t.da5 = (u32x4 *)take(T * slab);
    t.da4 = (u32x4 *)take(T * slab);
    t.dlat = (u32x4 *)take(2 * T * slab);
    t.da2 = (u32x4 *)take(2 * T * slab);
    t.da1 = (u32x4 *)take(2 * T * slab);
    t.gy = (float *)take(T * 32 * 4);
    t.dh0 = (float *)take(2 * B * kK0 * 4);
    t.partial = (double *)take(kFusedBlocksMax * 8);
    t.bytes = pos;
    return t;
}

static unsigned fused_blocks(int64_t B) {
    const int64_t b = ceil_div(ceil_div(B, 32), kTW);
    return (unsigned)(b < kFusedBlocksMax ? (b > 0 ? b : 1) : kFusedBlocksMax);
}

static FusedArgs fused_args(const ndf_net_config *c, const NetOffsets &o, const float *P,
                            const int64_t *pairs, const float *pos, const float *targets,
                            int64_t B, const FusedWS &t, float *y) {
    FusedArgs a{};
    a.P = P;
    for (int l = 0; l < kL; ++l) a.grid[l] = o.grid[0][l];
    for (int L = 0; L < 5; ++L) {
        a.wf[L] = t.fr.f[L];
        a.wt[L] = t.fr.t[L];
    }
    a.b[0] = P + o.b1[0];
    a.b[1] = P + o.b2[0];
    a.b[2] = P + o.b3[0];
    a.b[3] = P + o.b4;
    a.b[4] = P + o.b5;
    a.w6 = P + o.w6;
    a.b6 = P + o.b6;
    a.g = grid_geom(c);
    a.pairs = pairs;
    a.pos = pos;
    a.targets = targets;
    a.B = B;
    a.inv_b = 1.f / (float)B;
    a.h0 = t.h0; a.h1 = t.h1; a.h2 = t.h2; a.m = t.m; a.d1 = t.d1; a.d2 = t.d2;
    a.da5 = t.da5; a.da4 = t.da4; a.dlat = t.dlat; a.da2 = t.da2; a.da1 = t.da1;
    a.lat = t.lat;
    a.gy = t.gy;
    a.y = y;
    a.dh0 = t.dh0;
    a.partial = t.partial;
    return a;
}

static void fused_forward(const ndf_net_config *c, const NetOffsets &o, const float *P,
                          const int64_t *pairs, const float *pos, const float *targets, int64_t B,
                          const FusedWS &t, float *y, hipStream_t st) {
    hipLaunchKernelGGL(pack_train_kernel, dim3(64), dim3(256), 0, st, P, o.W1[0], o.W2[0],
                       o.W3[0], o.W4, o.W5, enc_in(c), t.fr);
    const FusedArgs a = fused_args(c, o, P, pairs, pos, targets, B, t, y);
    const dim3 g(fused_blocks(B)), b(kTThreads);
    if (c->fourier) {
        if (pos)
            hipLaunchKernelGGL((train_fwd_kernel<true, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((train_fwd_kernel<false, true>), g, b, 0, st, a);
    } else {
        if (pos)
            hipLaunchKernelGGL((train_fwd_kernel<true, false>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((train_fwd_kernel<false, false>), g, b, 0, st, a);
    }
}

static int fused_grad(const ndf_net_config *c, const float *P, const int64_t *pairs,
                      const float *pos, const float *targets, int64_t B, float *G, float *loss,
                      void *ws, hipStream_t st) {
    const NetOffsets o = net_offsets(c);
    const FusedWS t = carve_fused(c, ws, B);
    launch_status_clear(t.status, st);
    hipLaunchKernelGGL(fill_kernel, dim3(gs_blocks(o.total)), dim3(kThreads), 0, st, G, o.total,
                       0.f);
    fused_forward(c, o, P, pairs, pos, targets, B, t, nullptr, st);
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(64), 0, st, t.partial,
                       (int)fused_blocks(B), B, loss, t.status);
    const FusedArgs a = fused_args(c, o, P, pairs, pos, targets, B, t, nullptr);
    hipLaunchKernelGGL(train_bwd_kernel, dim3(fused_blocks(B)), dim3(kTThreads), 0, st, a);
    const int64_t rows = 2 * B;
    hipLaunchKernelGGL(grid_bwd_kernel, dim3((unsigned)grid_bwd_blocks(rows)), dim3(kThreads), 0,
                       st, G, grid_offs(o), grid_geom(c), 1, pairs, pos, B, (int64_t)0, rows,
                       t.dh0);
    WgradArgs w{};
    const int64_t T = ceil_div(B, 32);
    const u32x4 *gs[5] = {t.da1, t.da2, t.dlat, t.da4, t.da5};
    const u32x4 *xs[5] = {t.h0, t.h1, t.h2, t.m, t.d1};
    const int64_t ns[6] = {2 * T, 2 * T, 2 * T, T, T, T};
    float *dws[6] = {G + o.W1[0], G + o.W2[0], G + o.W3[0], G + o.W4, G + o.W5, G + o.w6};
    float *dbs[6] = {G + o.b1[0], G + o.b2[0], G + o.b3[0], G + o.b4, G + o.b5, G + o.b6};
    // workgroups per layer in proportion to the bytes it reads (per decoder slab:
    // W1 20 KB, W2 and W3 32, W4 and W5 16, the head 8), 511 in all, one round at
    // two workgroups per CU; at most one per slab pair
    const int share[6] = {82, 132, 132, 66, 66, 33};
    int acc_wg = 0;
    for (int L = 0; L < 6; ++L) {
        if (L < 5) {
            w.g[L] = gs[L];
            w.x[L] = xs[L];
        }
        w.nslab[L] = ns[L];
        w.dW[L] = dws[L];
        w.db[L] = dbs[L];
        w.wg0[L] = acc_wg;
        const int64_t pairs_l = ceil_div(ns[L], 2);
        acc_wg += (int)(pairs_l < share[L] ? pairs_l : share[L]);
    }
    w.wg0[6] = acc_wg;
    w.d2 = t.d2;
    w.gy = t.gy;
    w.kin1 = enc_in(c);
    hipLaunchKernelGGL(wgrad_all_kernel, dim3((unsigned)acc_wg), dim3(512), 0, st, w);
    return status_of_launch();
}

}  // namespace

size_t net_train_ws_bytes(const ndf_net_config *c, int64_t B) {
    return fused_path(c) ? carve_fused(c, nullptr, B).bytes : carve(nullptr, B).bytes;
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
        uni(o.W1[e], kH * enc_in(c), sqrtf(6.f / (float)enc_in(c)));
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
    if (fused_path(c)) {
        fused_forward(c, o, params, pairs, pos, nullptr, B, carve_fused(c, ws, B), y, st);
        return status_of_launch();
    }
    TrainWS t = carve(ws, B);
    t.y = y;
    forward(c, o, params, pairs, pos, nullptr, B, t, st);
    return status_of_launch();
}

int launch_net_grad(const ndf_net_config *c, const float *P, const int64_t *pairs,
                    const float *pos, const float *targets, int64_t B, float *G, float *loss,
                    void *ws, hipStream_t st) {
    if (fused_path(c)) return fused_grad(c, P, pairs, pos, targets, B, G, loss, ws, st);
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
            const int64_t gb = grid_bwd_blocks(rows);
            hipLaunchKernelGGL(grid_bwd_kernel, dim3((unsigned)gb),
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
        const int64_t gb = grid_bwd_blocks(rows);
        hipLaunchKernelGGL(grid_bwd_kernel, dim3((unsigned)gb),
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
