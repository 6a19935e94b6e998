// KSG targets at continuous positions (Sec. 4.3: training pairs are positions
// in the domain, the ensemble sampled there by trilinear interpolation).
//
// points_codes_kernel turns each interpolated column into a column of integer
// codes exactly as ndf_prepare does for a vertex (min-max onto [0, 2^23], IEEE
// double, round-half-even): column b is p1 of pair b (variable a), column B + b
// is p2 (variable b).  The samples are sum_c w_c x_m(v_c) over the corners of
// nonzero weight in corner order, in FP64 without contraction, so the codes are
// reproducible bit for bit; at a vertex's own position they equal that vertex's
// codes.  One wave per column reads its eight corner rows of the vertex-major
// copy once (16-byte loads when N % 4 == 0) and keeps the column's samples in
// registers (N <= 2048: 32 per lane) for the min/max and the coding pass.  The
// sorted-order kernel of ndf_prepare then sorts the 2B columns once each, and the
// KSG pairs kernel runs on them with pairs (b, B + b) exactly as on vertices.
#include "common.hpp"

#pragma clang fp contract(off)

namespace ndf {

int launch_ksg_pairs(const ndf_ensemble *e, int var_a, int var_b, const int64_t *pairs, int64_t B,
                     int k, float *out, int32_t *counts, double *H, hipStream_t st);
int launch_ksg_orders(const ndf_ensemble *e, hipStream_t st);
size_t ksg_pairs_ws_bytes(int N);

constexpr int kPtsPerLane = 32;  // 2048 members / 64 lanes

template <bool VEC>
__global__ __launch_bounds__(256) void points_codes_kernel(
    const float *__restrict__ xt_a, const float *__restrict__ xt_b, int N, int nx, int ny,
    int nz, const float *__restrict__ pos, int64_t B, int32_t *__restrict__ code,
    int32_t *__restrict__ flags, int64_t *__restrict__ pairs) {
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= 2 * B) return;
    const int side = col >= B ? 1 : 0;
    const int64_t b = col - side * B;
    const float *xt = side ? xt_b : xt_a;
    int64_t v[8];
    double w[8];
    data_cell(pos + 6 * b + 3 * side, nx, ny, nz, v, w);
    // member of slot i of this lane: 4 consecutive members per 16-byte load
    // (VEC), else one member per slot
    auto member = [&](int i) { return VEC ? 256 * (i >> 2) + 4 * lane + (i & 3) : 64 * i + lane; };
    double a[kPtsPerLane];
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < kPtsPerLane; i += (VEC ? 4 : 1)) {
        if (member(i) < N) {
            f32x4 xc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (VEC) {
                    xc[c] = *reinterpret_cast<const f32x4 *>(xt + v[c] * N + member(i));
                } else {
                    xc[c][0] = xt[v[c] * N + member(i)];
                }
            }
#pragma unroll
            for (int e = 0; e < (VEC ? 4 : 1); ++e) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (w[c] != 0.0) s += w[c] * (double)xc[c][e];
                a[i + e] = s;
                bad |= !isfinite(s);
                lo = fmin(lo, s);
                hi = fmax(hi, s);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    const bool flat = !(hi > lo);
    const double scale = flat ? 0.0 : 8388608.0 / (hi - lo);
    int32_t *dst = code + col * N;
#pragma unroll
    for (int i = 0; i < kPtsPerLane; i += (VEC ? 4 : 1)) {
        if (member(i) < N) {
            if (VEC) {
                i32x4 q;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    q[e] = (flat || bad) ? 0 : (int32_t)__builtin_rint((a[i + e] - lo) * scale);
                *reinterpret_cast<i32x4 *>(dst + member(i)) = q;
            } else {
                dst[member(i)] = (flat || bad) ? 0 : (int32_t)__builtin_rint((a[i] - lo) * scale);
            }
        }
    }
    if (lane == 0) {
        flags[col] = (bad ? NDF_FLAG_NONFINITE : 0) | (flat ? NDF_FLAG_CONSTANT : 0);
        if (!side) {
            pairs[2 * b] = b;
            pairs[2 * b + 1] = B + b;
        }
    }
}

size_t ksg_points_ws_bytes(int N, int64_t B) {
    return ksg_pairs_ws_bytes(N) + align_up((size_t)B * 2 * sizeof(int64_t), 256) +
           align_up((size_t)B * 2 * sizeof(int32_t), 256) +
           align_up((size_t)B * 2 * N * sizeof(int32_t), 256) +
           align_up((size_t)B * 2 * N * sizeof(uint16_t), 256);
}

int launch_ksg_points(const ndf_ensemble *e, int var_a, int var_b, const float *pos, int64_t B,
                      int k, float *out, int32_t *counts, void *ws, hipStream_t st) {
    const int N = e->n_members;
    if (N > 64 * kPtsPerLane) return NDF_E_UNSUPPORTED;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    char *w = (char *)ws;
    double *H = (double *)w;
    w += ksg_pairs_ws_bytes(N);
    int64_t *pairs = (int64_t *)w;
    w += align_up((size_t)B * 2 * sizeof(int64_t), 256);
    int32_t *flags = (int32_t *)w;
    w += align_up((size_t)B * 2 * sizeof(int32_t), 256);
    int32_t *code = (int32_t *)w;
    w += align_up((size_t)B * 2 * N * sizeof(int32_t), 256);
    uint16_t *order = (uint16_t *)w;
    const float *xa = e->xt + (int64_t)var_a * V * N, *xb = e->xt + (int64_t)var_b * V * N;
    const dim3 g((unsigned)ceil_div(2 * B, 4));
    if (N % 4 == 0)
        hipLaunchKernelGGL(points_codes_kernel<true>, g, dim3(256), 0, st, xa, xb, N, e->nx, e->ny,
                           e->nz, pos, B, code, flags, pairs);
    else
        hipLaunchKernelGGL(points_codes_kernel<false>, g, dim3(256), 0, st, xa, xb, N, e->nx,
                           e->ny, e->nz, pos, B, code, flags, pairs);
    // the 2B columns as a one-variable ensemble of 2B "vertices" with their orders
    ndf_ensemble cols = *e;
    cols.n_vars = 1;
    cols.nx = (int32_t)(2 * B);
    cols.ny = 1;
    cols.nz = 1;
    cols.code = code;
    cols.flags = flags;
    cols.order = order;
    const int s = launch_ksg_orders(&cols, st);
    if (s != NDF_OK) return s;
    return launch_ksg_pairs(&cols, 0, 0, pairs, B, k, out, counts, H, st);
}

}  // namespace ndf
