// Per-vertex standardisation statistics and KSG integer codes.
//
// Pearson's r (Sec. 3.1, Eq. 1) needs per-vertex means and variances; the KSG
// estimator (Sec. 3.2) compares samples under the max-norm, for which every
// vertex is mapped onto integer codes in [0, 2^23] by min-max normalisation.
// The codes use only correctly rounded IEEE double operations (subtract,
// multiply, divide) and round-half-even, so they are the same integers on any
// conforming implementation; all later KSG distances are exact int32.
//
// One workgroup owns 64 consecutive vertices of one variable.  The ensemble is
// member-major, so each member row contributes a 256-byte coalesced segment.
// Codes are written vertex-major through an LDS transpose (64 members x 64
// vertices per tile).
#include "common.hpp"

#pragma clang fp contract(off)

namespace ndf {

constexpr int kPrepV = 64;          // vertices per workgroup
constexpr int kPrepPh = 4;          // member phases per vertex
constexpr int kPrepThreads = kPrepV * kPrepPh;

__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(
    const float *__restrict__ x, int N, int64_t V, double *__restrict__ mean,
    double *__restrict__ inv_std, int32_t *__restrict__ code, int32_t *__restrict__ flags) {
    const int var = blockIdx.y;
    const float *xv = x + (int64_t)var * N * V;
    const int t = threadIdx.x;
    const int vl = t % kPrepV;
    const int ph = t / kPrepV;
    const int64_t v0 = (int64_t)blockIdx.x * kPrepV;
    const int64_t v = v0 + vl;
    const bool live = v < V;

    __shared__ double s_sum[kPrepPh][kPrepV];
    __shared__ float s_lo[kPrepPh][kPrepV];
    __shared__ float s_hi[kPrepPh][kPrepV];
    __shared__ int s_bad[kPrepPh][kPrepV];
    __shared__ int32_t s_tile[64][kPrepV + 1];

    // pass 1: sum, min, max, finiteness
    double sum = 0.0;
    float lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    if (live) {
        for (int m = ph; m < N; m += kPrepPh) {
            float a = xv[(int64_t)m * V + v];
            sum += (double)a;
            lo = fminf(lo, a);
            hi = fmaxf(hi, a);
            bad |= !isfinite(a);
        }
    }
    s_sum[ph][vl] = sum;
    s_lo[ph][vl] = lo;
    s_hi[ph][vl] = hi;
    s_bad[ph][vl] = bad;
    __syncthreads();
    sum = 0.0;
    lo = INFINITY;
    hi = -INFINITY;
    bad = 0;
    for (int p = 0; p < kPrepPh; ++p) {
        sum += s_sum[p][vl];
        lo = fminf(lo, s_lo[p][vl]);
        hi = fmaxf(hi, s_hi[p][vl]);
        bad |= s_bad[p][vl];
    }
    const double mu = sum / (double)N;
    __syncthreads();

    // pass 2: centred sum of squares
    double ss = 0.0;
    if (live) {
        for (int m = ph; m < N; m += kPrepPh) {
            double d = (double)xv[(int64_t)m * V + v] - mu;
            ss += d * d;
        }
    }
    s_sum[ph][vl] = ss;
    __syncthreads();
    ss = 0.0;
    for (int p = 0; p < kPrepPh; ++p) ss += s_sum[p][vl];
    const bool flat = !(hi > lo);
    if (live && ph == 0) {
        const double var_pop = ss / (double)N;
        mean[(int64_t)var * V + v] = mu;
        inv_std[(int64_t)var * V + v] = (var_pop > 0.0 && !flat) ? 1.0 / sqrt(var_pop) : 0.0;
        flags[(int64_t)var * V + v] = (bad ? NDF_FLAG_NONFINITE : 0) | (flat ? NDF_FLAG_CONSTANT : 0);
    }

    // pass 3: codes, transposed through LDS into vertex-major rows
    const double dlo = (double)lo;
    const double scale = flat ? 0.0 : 8388608.0 / ((double)hi - dlo);
    int32_t *cv = code + (int64_t)var * V * N;
    for (int m0 = 0; m0 < N; m0 += 64) {
        for (int mm = ph; mm < 64; mm += kPrepPh) {
            const int m = m0 + mm;
            int32_t c = 0;
            if (live && m < N && !flat) {
                double tq = ((double)xv[(int64_t)m * V + v] - dlo) * scale;
                c = (int32_t)__builtin_rint(tq);
            }
            s_tile[mm][vl] = c;
        }
        __syncthreads();
        // 64 rows (vertices) of up to 64 members; 16 threads per row, 4 members each
        for (int pass = 0; pass < 4; ++pass) {
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
}

int launch_prepare(const ndf_ensemble *e, hipStream_t st) {
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    dim3 grid((unsigned)ceil_div(V, kPrepV), (unsigned)e->n_vars);
    hipLaunchKernelGGL(prepare_kernel, grid, dim3(kPrepThreads), 0, st, e->x, e->n_members, V,
                       e->mean, e->inv_std, e->code, e->flags);
    return status_of_launch();
}

}  // namespace ndf
