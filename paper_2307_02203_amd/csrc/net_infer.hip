// Learned dependence field inference (Sec. 5): phi(p) = Phi(p_ref, p) at every
// grid vertex, in one fused kernel per reference.
//
// The reference latent is computed once (same kernel, latent-only mode).  Each
// wave then takes 64 query vertices at a time through
//   grid gather (4 levels x 8 corners of 8 bf16 features, FP32 trilinear weights)
//   -> L1 32->128 ReLU -> L2 128->128 ReLU -> L3 128->128 (latent)
//   -> product with the reference latent -> L4 ReLU -> L5 ReLU -> w6 . d2 + b6
// entirely in registers: every layer is MFMA 32x32x16 bf16 with FP32 accumulate,
// the weights of all layers (136 KB bf16) sit in LDS for the whole launch in
// MFMA operand order, and a layer's FP32 accumulators are rounded to bf16 and
// used directly as the next layer's B operand.  That works because the MFMA
// output layout (lane = query, 16 feature rows per lane) equals the operand
// layout up to a fixed permutation of the contraction index inside every
// 16-block, which is folded into the packed weights:
//   logical k = 16 kb + 8 h + e  <->  feature 16 kb + 8 (e / 4) + 4 h + e % 4.
// Latents are rounded to bf16 before the product, and the product of two bf16
// numbers is exact in FP32, so Phi(p, q) and Phi(q, p) of a self field are
// computed identically.
#include "net.hpp"

namespace ndf {

constexpr int kInferWaves = 8;
constexpr int kInferThreads = 64 * kInferWaves;

// Byte offsets inside the packed inference parameters.
struct QLayout {
    int64_t grid[2][kL];           // bf16 [cells][8]
    int64_t w1[2], w2[2], w3[2];   // bf16 MFMA A fragments
    int64_t w4, w5;
    int64_t b1[2], b2[2], b3[2];   // fp32 [128]
    int64_t b4, b5, w6, b6;        // fp32
    int64_t total;
};

static QLayout qlayout(const ndf_net_config *c) {
    QLayout q{};
    int64_t pos = 0;
    auto take = [&](int64_t bytes) {
        int64_t at = pos;
        pos += (int64_t)align_up((size_t)bytes, 256);
        return at;
    };
    const NetOffsets o = net_offsets(c);
    for (int e = 0; e < c->n_enc; ++e) {
        for (int l = 0; l < kL; ++l) q.grid[e][l] = take(o.cells[l] * kF * 2);
        q.w1[e] = take(kH * kK0 * 2);
        q.w2[e] = take(kH * kH * 2);
        q.w3[e] = take(kH * kH * 2);
        q.b1[e] = take(kH * 4);
        q.b2[e] = take(kH * 4);
        q.b3[e] = take(kH * 4);
    }
    if (c->n_enc == 1) {
        for (int l = 0; l < kL; ++l) q.grid[1][l] = q.grid[0][l];
        q.w1[1] = q.w1[0]; q.w2[1] = q.w2[0]; q.w3[1] = q.w3[0];
        q.b1[1] = q.b1[0]; q.b2[1] = q.b2[0]; q.b3[1] = q.b3[0];
    }
    q.w4 = take(kH * kH * 2);
    q.w5 = take(kH * kH * 2);
    q.b4 = take(kH * 4);
    q.b5 = take(kH * 4);
    q.w6 = take(kH * 4);
    q.b6 = take(4);
    q.total = pos;
    return q;
}

size_t net_qparam_bytes(const ndf_net_config *c, int prec) {
    (void)prec;
    return (size_t)qlayout(c).total;
}

size_t net_infer_ws_bytes(const ndf_net_config *c, int64_t n_ref, int prec) {
    (void)c;
    (void)prec;
    return align_up((size_t)n_ref * kH * sizeof(float), 256) +
           align_up((size_t)n_ref * sizeof(int64_t), 256);
}

// ----------------------------------------------------------- quantize ----
__global__ void to_bf16_kernel(const float *__restrict__ src, int64_t n,
                               uint16_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f2bf_bits(src[i]);
}

// A fragments of W[128][KIN] (row-major): frag[(ob*KB + kb)*64 + lane][e] =
// W[32 ob + lane%32][k], k natural (first layer) or permuted to match the
// previous layer's output layout.
__global__ void pack_frag_kernel(const float *__restrict__ W, int KIN, int permuted,
                                 uint16_t *__restrict__ frag) {
    const int KB = KIN / 16;
    const int n = kH * KIN;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int e = t & 7;
        const int lane = (t >> 3) & 63;
        const int fi = t >> 9;  // fragment index ob*KB + kb
        const int ob = fi / KB, kb = fi % KB;
        const int h = lane >> 5, il = lane & 31;
        const int k = permuted ? 16 * kb + 8 * (e >> 2) + 4 * h + (e & 3) : 16 * kb + 8 * h + e;
        frag[t] = f2bf_bits(W[(32 * ob + il) * KIN + k]);
    }
}

__global__ void copy_f32_kernel(const float *__restrict__ src, int n, float *__restrict__ dst) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int launch_net_quantize(const ndf_net_config *c, const float *P, int prec, void *qp,
                        hipStream_t st) {
    if (prec != NDF_PREC_BF16) return NDF_E_UNSUPPORTED;
    const NetOffsets o = net_offsets(c);
    const QLayout q = qlayout(c);
    char *Q = (char *)qp;
    for (int e = 0; e < c->n_enc; ++e) {
        for (int l = 0; l < kL; ++l) {
            const int64_t n = o.cells[l] * kF;
            int64_t nb = ceil_div(n, 256);
            hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256),
                               0, st, P + o.grid[e][l], n, (uint16_t *)(Q + q.grid[e][l]));
        }
        hipLaunchKernelGGL(pack_frag_kernel, dim3(16), dim3(256), 0, st, P + o.W1[e], kK0, 0,
                           (uint16_t *)(Q + q.w1[e]));
        hipLaunchKernelGGL(pack_frag_kernel, dim3(64), dim3(256), 0, st, P + o.W2[e], kH, 1,
                           (uint16_t *)(Q + q.w2[e]));
        hipLaunchKernelGGL(pack_frag_kernel, dim3(64), dim3(256), 0, st, P + o.W3[e], kH, 1,
                           (uint16_t *)(Q + q.w3[e]));
        hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.b1[e], kH,
                           (float *)(Q + q.b1[e]));
        hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.b2[e], kH,
                           (float *)(Q + q.b2[e]));
        hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.b3[e], kH,
                           (float *)(Q + q.b3[e]));
    }
    hipLaunchKernelGGL(pack_frag_kernel, dim3(64), dim3(256), 0, st, P + o.W4, kH, 1,
                       (uint16_t *)(Q + q.w4));
    hipLaunchKernelGGL(pack_frag_kernel, dim3(64), dim3(256), 0, st, P + o.W5, kH, 1,
                       (uint16_t *)(Q + q.w5));
    hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.b4, kH,
                       (float *)(Q + q.b4));
    hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.b5, kH,
                       (float *)(Q + q.b5));
    hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(128), 0, st, P + o.w6, kH,
                       (float *)(Q + q.w6));
    hipLaunchKernelGGL(copy_f32_kernel, dim3(1), dim3(1), 0, st, P + o.b6, 1, (float *)(Q + q.b6));
    return status_of_launch();
}

// ------------------------------------------------------- fused kernel ----
struct InferArgs {
    const uint16_t *grid[kL];   // bf16 [cells][8] of the query encoder
    const bf16x8 *w[5];         // A fragments W1..W5
    const float *b[5];          // b1..b5
    const float *w6;
    const float *b6;
    GridGeom g;
    int64_t V;
};

// LDS plan (bytes): W1 8K | W2..W5 4 x 32K | b1..b5 5 x 512 | w6 512 | ref latent 512
constexpr int kFragW1 = 4 * 2 * 64;   // bf16x8 elements
constexpr int kFragW = 4 * 8 * 64;

// Corner cells (int32) and weights of vertex v on level l; same arithmetic as
// the training lookup.
__device__ __forceinline__ void corners32(const GridGeom &g, const int R[3], int64_t v, int idx[8],
                                          float w[8]) {
    int64_t i64[8];
    corners_R(g, R, v, i64, w);
#pragma unroll
    for (int c = 0; c < 8; ++c) idx[c] = (int)i64[c];
}

enum { LAY_RELU = 0, LAY_LATENT = 1, LAY_HEAD = 2, LAY_LATENT_OUT = 3 };

// One 128-wide layer for the wave's 2 x 32 queries.  in: KB k-blocks of B
// operands; per output block ob the two accumulators (one per query block) are
// finished and turned into out[2 ob], out[2 ob + 1] (or the head / latent).
template <int KB, int KIND>
__device__ __forceinline__ void dense_layer(const bf16x8 *__restrict__ wf,
                                            const float *__restrict__ bias,
                                            const float *__restrict__ ref,
                                            const float *__restrict__ w6,
                                            const bf16x8 (&in)[8][2], bf16x8 (&out)[8][2],
                                            float (&part)[2], float *__restrict__ lat_out,
                                            int64_t row0, const bool (&ok)[2], int lane, int h4) {
    // per-lane row offset 4*(lane/32); rows of block ob are h4 + 32 ob + 8 (r/4) + r%4
    const float *bias_h = bias + h4;
    const float *ref_h = ref + h4;
    const float *w6_h = w6 + h4;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x16 acc0, acc1;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.f;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const bf16x8 a = wf[(ob * KB + kb) * 64 + lane];
            acc0 = mfma32(a, in[kb][0], acc0);
            acc1 = mfma32(a, in[kb][1], acc1);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            bf16x8 t0, t1;  // built whole, so the previous contents of out[] die here
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = 8 * s + e;
                const int i = 32 * ob + d_row(r, lane);
                const int ic = 32 * ob + 8 * (r >> 2) + (r & 3);  // i - h4, compile-time
                const float bi = bias_h[ic];
                float v0 = acc0[r] + bi, v1 = acc1[r] + bi;
                if (KIND == LAY_RELU || KIND == LAY_HEAD) {
                    v0 = v0 > 0.f ? v0 : 0.f;
                    v1 = v1 > 0.f ? v1 : 0.f;
                }
                if (KIND == LAY_LATENT || KIND == LAY_LATENT_OUT) {
                    v0 = bf2f(f2bf(v0));  // latent rounded to bf16
                    v1 = bf2f(f2bf(v1));
                }
                if (KIND == LAY_LATENT_OUT) {
                    if (ok[0]) lat_out[(row0 + (lane & 31)) * kH + i] = v0;
                    if (ok[1]) lat_out[(row0 + 32 + (lane & 31)) * kH + i] = v1;
                } else if (KIND == LAY_HEAD) {
                    part[0] = fmaf(w6_h[ic], v0, part[0]);
                    part[1] = fmaf(w6_h[ic], v1, part[1]);
                } else {
                    if (KIND == LAY_LATENT) {  // product with the reference latent: exact in FP32
                        v0 *= ref_h[ic];
                        v1 *= ref_h[ic];
                    }
                    t0[e] = f2bf(v0);
                    t1[e] = f2bf(v1);
                }
            }
            if (KIND == LAY_RELU || KIND == LAY_LATENT) {
                out[2 * ob + s][0] = t0;
                out[2 * ob + s][1] = t1;
            }
        }
        // keep the scheduler from hoisting the next block's operand loads above
        // this epilogue (that would hold ~128 extra registers)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// MODE 0: field (out[v] = Phi(ref, v) for v < nq); MODE 1: latents of the
// vertices in qlist (lat_out[n][128], bf16-rounded values stored as FP32).
template <int MODE>
__global__ __launch_bounds__(kInferThreads) void infer_kernel(InferArgs A,
                                                              const int64_t *__restrict__ qlist,
                                                              int64_t nq,
                                                              const float *__restrict__ ref_lat,
                                                              float *__restrict__ out) {
    __shared__ bf16x8 s_w1[kFragW1];
    __shared__ bf16x8 s_w[4][kFragW];
    __shared__ float s_b[5][kH];
    __shared__ float s_w6[kH];
    __shared__ float s_ref[kH];

    const int tid = threadIdx.x;
    for (int i = tid; i < kFragW1; i += kInferThreads) s_w1[i] = A.w[0][i];
    const int nlay = MODE == 0 ? 4 : 2;  // latent mode needs W2, W3 only
    for (int L = 0; L < nlay; ++L)
        for (int i = tid; i < kFragW; i += kInferThreads) s_w[L][i] = A.w[L + 1][i];
    for (int i = tid; i < 5 * kH; i += kInferThreads) s_b[i / kH][i % kH] = A.b[i / kH][i % kH];
    for (int i = tid; i < kH; i += kInferThreads) {
        s_w6[i] = A.w6[i];
        s_ref[i] = MODE == 0 ? ref_lat[i] : 0.f;
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, jl = lane & 31;
    const float b6 = A.b6[0];
    const int64_t ntiles = ceil_div(nq, 64);
    for (int64_t tile = (int64_t)blockIdx.x * kInferWaves + wave; tile < ntiles;
         tile += (int64_t)gridDim.x * kInferWaves) {
        const int64_t row0 = tile * 64;
        // opaque per tile, so the per-lane LDS addresses derived from it are
        // formed inside the loop (base + immediate) instead of hoisted and spilled
        int h4 = 4 * h;
        asm volatile("" : "+v"(h4));
        bool ok[2];
        int64_t vq[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t n = row0 + q * 32 + jl;
            ok[q] = n < nq;
            vq[q] = ok[q] ? (qlist ? qlist[n] : n) : 0;
        }
        // grid gather: k-block kb, half h -> level 2 kb + h (its 8 features)
        bf16x8 a[8][2], b[8][2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            // both candidate levels are uniform; the lane half picks one
            const uint16_t *grid = h ? A.grid[2 * kb + 1] : A.grid[2 * kb];
            int R[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) R[ax] = h ? A.g.R[2 * kb + 1][ax] : A.g.R[2 * kb][ax];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                int idx[8];
                float w[8];
                corners32(A.g, R, vq[q], idx, w);
                float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int cn = 0; cn < 8; ++cn) {
                    const i32x4 raw = *reinterpret_cast<const i32x4 *>(grid + (int64_t)idx[cn] * kF);
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const uint32_t u = (uint32_t)raw[p];
                        s[2 * p] = fmaf(w[cn], __uint_as_float(u << 16), s[2 * p]);
                        s[2 * p + 1] = fmaf(w[cn], __uint_as_float(u & 0xffff0000u), s[2 * p + 1]);
                    }
                }
                bf16x8 t;
#pragma unroll
                for (int e = 0; e < 8; ++e) t[e] = f2bf(s[e]);
                a[kb][q] = t;
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        float part[2] = {0.f, 0.f};
        dense_layer<2, LAY_RELU>(s_w1, s_b[0], s_ref, s_w6, a, b, part, nullptr, row0, ok, lane, h4);
        dense_layer<8, LAY_RELU>(s_w[0], s_b[1], s_ref, s_w6, b, a, part, nullptr, row0, ok, lane, h4);
        if (MODE == 1) {
            dense_layer<8, LAY_LATENT_OUT>(s_w[1], s_b[2], s_ref, s_w6, a, b, part, out, row0, ok,
                                           lane, h4);
            continue;
        }
        dense_layer<8, LAY_LATENT>(s_w[1], s_b[2], s_ref, s_w6, a, b, part, nullptr, row0, ok,
                                   lane, h4);
        dense_layer<8, LAY_RELU>(s_w[2], s_b[3], s_ref, s_w6, b, a, part, nullptr, row0, ok, lane, h4);
        dense_layer<8, LAY_HEAD>(s_w[3], s_b[4], s_ref, s_w6, a, b, part, nullptr, row0, ok, lane, h4);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float y = part[q] + __shfl_xor(part[q], 32, 64) + b6;
            if (h == 0 && ok[q]) out[row0 + q * 32 + jl] = y;
        }
    }
}

static InferArgs make_args(const ndf_net_config *c, const QLayout &q, const char *Q, int e) {
    InferArgs a{};
    for (int l = 0; l < kL; ++l) a.grid[l] = (const uint16_t *)(Q + q.grid[e][l]);
    a.w[0] = (const bf16x8 *)(Q + q.w1[e]);
    a.w[1] = (const bf16x8 *)(Q + q.w2[e]);
    a.w[2] = (const bf16x8 *)(Q + q.w3[e]);
    a.w[3] = (const bf16x8 *)(Q + q.w4);
    a.w[4] = (const bf16x8 *)(Q + q.w5);
    a.b[0] = (const float *)(Q + q.b1[e]);
    a.b[1] = (const float *)(Q + q.b2[e]);
    a.b[2] = (const float *)(Q + q.b3[e]);
    a.b[3] = (const float *)(Q + q.b4);
    a.b[4] = (const float *)(Q + q.b5);
    a.w6 = (const float *)(Q + q.w6);
    a.b6 = (const float *)(Q + q.b6);
    a.g = grid_geom(c);
    a.V = (int64_t)c->nx * c->ny * c->nz;
    return a;
}

static unsigned infer_blocks(int64_t nq) {
    const int64_t tiles = ceil_div(nq, 64);
    const int64_t b = ceil_div(tiles, kInferWaves);
    return (unsigned)(b < 256 ? (b > 0 ? b : 1) : 256);  // one resident workgroup per CU
}

int launch_infer_field(const ndf_net_config *c, const void *qp, int prec, const int64_t *ref_v,
                       int n_ref, float *out, void *ws, hipStream_t st) {
    if (prec != NDF_PREC_BF16) return NDF_E_UNSUPPORTED;
    const QLayout q = qlayout(c);
    const char *Q = (const char *)qp;
    float *lat = (float *)ws;
    int64_t *refs = (int64_t *)((char *)ws + align_up((size_t)n_ref * kH * sizeof(float), 256));
    if (hipMemcpyAsync(refs, ref_v, (size_t)n_ref * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return NDF_E_HIP;
    // reference latents with encoder 0 (p1), queries with the last encoder (p2)
    const InferArgs a0 = make_args(c, q, Q, 0);
    hipLaunchKernelGGL(infer_kernel<1>, dim3(infer_blocks(n_ref)), dim3(kInferThreads), 0, st, a0,
                       refs, (int64_t)n_ref, nullptr, lat);
    const InferArgs a1 = make_args(c, q, Q, c->n_enc - 1);
    const int64_t V = a1.V;
    for (int r = 0; r < n_ref; ++r)
        hipLaunchKernelGGL(infer_kernel<0>, dim3(infer_blocks(V)), dim3(kInferThreads), 0, st, a1,
                           nullptr, V, lat + (int64_t)r * kH, out + (int64_t)r * V);
    return status_of_launch();
}

}  // namespace ndf
