// Per-vertex standardisation statistics and KSG integer codes.
//
// Pearson's r (Sec. 3.1, Eq. 1) needs per-vertex means and variances; the KSG
// estimator (Sec. 3.2) compares samples under the max-norm, for which every
// vertex is mapped onto integer codes in [0, 2^23] by min-max normalisation.
// The codes use only correctly rounded IEEE double operations (subtract,
// multiply, divide) and round-half-even, so they are the same integers on any
// conforming implementation; all later KSG distances are exact int32.
//
// One workgroup owns 64 consecutive vertices of one variable and reads their
// members twice (sum / min / max, then centred squares and codes).  The ensemble
// is member-major, so each member row contributes a 256-byte coalesced segment.
// Codes are written vertex-major through an LDS transpose (64 members x 64
// vertices per tile).  Each thread keeps 8 (first pass) or 16 (second pass) of
// its member loads in flight; one load at a time left the kernel latency-bound at
// 3.3 TB/s.  (Two vertices per thread with 8-byte loads measured slower: the
// larger tile cut the resident workgroups per CU.)
#include "common.hpp"

#pragma clang fp contract(off)

namespace ndf {

constexpr int kPrepVW = 1;                    // consecutive vertices per thread (1 or 2)
constexpr int kPrepG = 64;                    // vertex groups per workgroup
constexpr int kPrepV = kPrepG * kPrepVW;      // vertices per workgroup
constexpr int kPrepPh = 4;                    // member phases per vertex group
constexpr int kPrepThreads = kPrepG * kPrepPh;

__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(
    const float *__restrict__ x, int N, int64_t V, double *__restrict__ mean,
    double *__restrict__ inv_std, int32_t *__restrict__ code, int32_t *__restrict__ flags,
    int32_t *__restrict__ status) {
    const int var = blockIdx.y;
    const float *xv = x + (int64_t)var * N * V;
    const int t = threadIdx.x;
    const int vg = t % kPrepG;
    const int ph = t / kPrepG;
    const int64_t v0 = (int64_t)blockIdx.x * kPrepV;
    const int64_t vb = v0 + kPrepVW * vg;  // this thread's first vertex
    // 8-byte loads need V even (every member row then starts 8-byte aligned)
    const bool pairs = (V % 2) == 0;

    __shared__ double s_sum[kPrepPh][kPrepV];
    __shared__ float s_lo[kPrepPh][kPrepV];
    __shared__ float s_hi[kPrepPh][kPrepV];
    __shared__ int s_bad[kPrepPh][kPrepV];
    __shared__ int32_t s_tile[64][kPrepV + 1];

    auto load = [&](int m, float (&a)[kPrepVW]) {
        const float *row = xv + (int64_t)m * V;
        if (kPrepVW == 2 && pairs && vb + 1 < V) {
            const f32x2 q = *reinterpret_cast<const f32x2 *>(row + vb);
            a[0] = q[0];
            a[1] = q[1];
        } else {
#pragma unroll
            for (int j = 0; j < kPrepVW; ++j) a[j] = vb + j < V ? row[vb + j] : 0.f;
        }
    };

    // pass 1: sum, min, max, finiteness
    double sum[kPrepVW];
    float lo[kPrepVW], hi[kPrepVW];
    int bad[kPrepVW];
#pragma unroll
    for (int j = 0; j < kPrepVW; ++j) {
        sum[j] = 0.0;
        lo[j] = INFINITY;
        hi[j] = -INFINITY;
        bad[j] = 0;
    }
    auto accumulate = [&](const float (&a)[kPrepVW]) {
#pragma unroll
        for (int j = 0; j < kPrepVW; ++j) {
            sum[j] += (double)a[j];
            lo[j] = fminf(lo[j], a[j]);
            hi[j] = fmaxf(hi[j], a[j]);
            bad[j] |= !isfinite(a[j]);
        }
    };
    if (vb < V) {
        // eight members' loads in flight at a time; the sums keep member order
        constexpr int U = 8;
        int m = ph;
        for (; m + kPrepPh * (U - 1) < N; m += kPrepPh * U) {
            float a[U][kPrepVW];
#pragma unroll
            for (int u = 0; u < U; ++u) load(m + kPrepPh * u, a[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) accumulate(a[u]);
        }
        for (; m < N; m += kPrepPh) {
            float a[kPrepVW];
            load(m, a);
            accumulate(a);
        }
    }
#pragma unroll
    for (int j = 0; j < kPrepVW; ++j) {
        const int vl = kPrepVW * vg + j;
        s_sum[ph][vl] = sum[j];
        s_lo[ph][vl] = lo[j];
        s_hi[ph][vl] = hi[j];
        s_bad[ph][vl] = bad[j];
    }
    __syncthreads();
    double mu[kPrepVW], dlo[kPrepVW], scale[kPrepVW];
    bool flat[kPrepVW];
#pragma unroll
    for (int j = 0; j < kPrepVW; ++j) {
        const int vl = kPrepVW * vg + j;
        double sm = 0.0;
        float l = INFINITY, h = -INFINITY;
        int b = 0;
        for (int p = 0; p < kPrepPh; ++p) {
            sm += s_sum[p][vl];
            l = fminf(l, s_lo[p][vl]);
            h = fmaxf(h, s_hi[p][vl]);
            b |= s_bad[p][vl];
        }
        mu[j] = sm / (double)N;
        flat[j] = !(h > l);
        dlo[j] = (double)l;
        scale[j] = flat[j] ? 0.0 : 8388608.0 / ((double)h - dlo[j]);
        bad[j] = b;
    }
    __syncthreads();

    // pass 2: centred sum of squares and the codes, transposed through LDS into
    // vertex-major rows.  A thread visits members ph, ph + 4, ... in increasing
    // order, so its FP64 sum is the plain two-pass one.
    int32_t *cv = code + (int64_t)var * V * N;
    double ss[kPrepVW];
#pragma unroll
    for (int j = 0; j < kPrepVW; ++j) ss[j] = 0.0;
    for (int m0 = 0; m0 < N; m0 += 64) {
        // the tile's 16 loads of this thread in flight together
        float at[64 / kPrepPh][kPrepVW];
#pragma unroll
        for (int i = 0; i < 64 / kPrepPh; ++i) {
            const int m = m0 + ph + kPrepPh * i;
            if (vb < V && m < N) load(m, at[i]);
        }
#pragma unroll
        for (int i = 0; i < 64 / kPrepPh; ++i) {
            const int mm = ph + kPrepPh * i;
            const int m = m0 + mm;
            const float (&a)[kPrepVW] = at[i];
#pragma unroll
            for (int j = 0; j < kPrepVW; ++j) {
                int32_t c = 0;
                if (vb + j < V && m < N) {
                    const double d = (double)a[j] - mu[j];
                    ss[j] += d * d;
                    if (!flat[j]) c = (int32_t)__builtin_rint(((double)a[j] - dlo[j]) * scale[j]);
                }
                s_tile[mm][kPrepVW * vg + j] = c;
            }
        }
        __syncthreads();
        // kPrepV rows (vertices) of up to 64 members; 16 threads per row, 4 members each
        for (int pass = 0; pass < kPrepV / 16; ++pass) {
            const int row = t / 16 + 16 * pass;
            const int c4 = t % 16;
            const int64_t vr = v0 + row;
            const int mb = m0 + 4 * c4;
            if (vr < V) {
                int32_t *dst = cv + vr * N + mb;
                if (mb + 3 < N && ((N & 3) == 0)) {
                    i32x4 q;
                    q.x = s_tile[4 * c4 + 0][row];
                    q.y = s_tile[4 * c4 + 1][row];
                    q.z = s_tile[4 * c4 + 2][row];
                    q.w = s_tile[4 * c4 + 3][row];
                    *reinterpret_cast<i32x4 *>(dst) = q;
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (mb + e < N) dst[e] = s_tile[4 * c4 + e][row];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kPrepVW; ++j) s_sum[ph][kPrepVW * vg + j] = ss[j];
    __syncthreads();
    if (ph == 0) {
#pragma unroll
        for (int j = 0; j < kPrepVW; ++j) {
            const int64_t v = vb + j;
            if (v >= V) continue;
            double s2 = 0.0;
            for (int p = 0; p < kPrepPh; ++p) s2 += s_sum[p][kPrepVW * vg + j];
            const double var_pop = s2 / (double)N;
            mean[(int64_t)var * V + v] = mu[j];
            inv_std[(int64_t)var * V + v] = (var_pop > 0.0 && !flat[j]) ? 1.0 / sqrt(var_pop) : 0.0;
            flags[(int64_t)var * V + v] =
                (bad[j] ? NDF_FLAG_NONFINITE : 0) | (flat[j] ? NDF_FLAG_CONSTANT : 0);
            // every writer stores the same value, so the unordered stores agree
            if (bad[j] && status) *status = NDF_E_NONFINITE;
        }
    }
}

// Vertex-major copy xt[v][m] of the member-major ensemble x[m][v] (for the
// reads of a few scattered vertices' full columns, as interpolation at
// continuous positions does): 64 x 64 tiles through LDS.  VEC (V and N multiples
// of 4): 16-byte loads of four vertices of a member row and 16-byte stores of
// four members of a vertex row, 16 threads per 256-byte row segment.
template <bool VEC>
__global__ __launch_bounds__(256) void transpose_kernel(const float *__restrict__ x, int N,
                                                        int64_t V, float *__restrict__ xt) {
    __shared__ float tile[64][65];
    const int var = blockIdx.z;
    const float *xv = x + (int64_t)var * N * V;
    float *tv = xt + (int64_t)var * V * N;
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int m0 = blockIdx.y * 64;
    if (VEC) {
        const int c4 = threadIdx.x & 15, r = threadIdx.x >> 4;  // 16 rows of 16 x 16 B
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + r + 16 * i;
            const int64_t v = v0 + 4 * c4;
            f32x4 q = {0.f, 0.f, 0.f, 0.f};
            if (m < N && v < V)
                q = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(xv + (int64_t)m * V + v));
#pragma unroll
            for (int e = 0; e < 4; ++e) tile[r + 16 * i][4 * c4 + e] = q[e];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int vl = r + 16 * i;
            const int64_t v = v0 + vl;
            const int m = m0 + 4 * c4;
            if (v < V && m < N) {
                f32x4 q;
#pragma unroll
                for (int e = 0; e < 4; ++e) q[e] = tile[4 * c4 + e][vl];
                *reinterpret_cast<f32x4 *>(tv + v * N + m) = q;
            }
        }
        return;
    }
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int m = m0 + i;
        const int64_t v = v0 + tx;
        tile[i][tx] = (m < N && v < V) ? __builtin_nontemporal_load(xv + (int64_t)m * V + v) : 0.f;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t v = v0 + i;
        const int m = m0 + tx;
        if (v < V && m < N) tv[v * N + m] = tile[tx][i];
    }
}

__global__ void status_clear_kernel(int32_t *status) { *status = NDF_OK; }

int launch_status_clear(int32_t *status, hipStream_t st) {
    hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(1), 0, st, status);
    return status_of_launch();
}

int launch_prepare(const ndf_ensemble *e, int32_t *status, hipStream_t st) {
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    if (status) launch_status_clear(status, st);
    dim3 grid((unsigned)ceil_div(V, kPrepV), (unsigned)e->n_vars);
    hipLaunchKernelGGL(prepare_kernel, grid, dim3(kPrepThreads), 0, st, e->x, e->n_members, V,
                       e->mean, e->inv_std, e->code, e->flags, status);
    if (e->xt) {
        dim3 tg((unsigned)ceil_div(V, 64), (unsigned)ceil_div(e->n_members, 64),
                (unsigned)e->n_vars);
        if (V % 4 == 0 && e->n_members % 4 == 0)
            hipLaunchKernelGGL(transpose_kernel<true>, tg, dim3(256), 0, st, e->x, e->n_members, V,
                               e->xt);
        else
            hipLaunchKernelGGL(transpose_kernel<false>, tg, dim3(256), 0, st, e->x, e->n_members,
                               V, e->xt);
    }
    return status_of_launch();
}

}  // namespace ndf
