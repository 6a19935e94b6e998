// Shared device helpers of the gfx950 kernels: bf16/fp8 conversions, MFMA
// operand types, wave reductions and launch bookkeeping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ndf.h"

namespace ndf {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) int i32x4;

constexpr int kWave = 64;

// MFMA 32x32x16 (bf16 in, fp32 accumulate), one wave:
//   A operand: lane l holds A[i = l%32][k = 8*(l/32) + e], e = 0..7
//   B operand: lane l holds B[k = 8*(l/32) + e][j = l%32]
//   D        : lane l, register r holds D[i = 8*(r/4) + 4*(l/32) + r%4][j = l%32]
__device__ __forceinline__ f32x16 mfma32(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int d_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// float -> bf16, round to nearest even (one v_cvt_pk_bf16_f32 per pair on gfx950).
__device__ __forceinline__ __bf16 f2bf(float f) { return static_cast<__bf16>(f); }
__device__ __forceinline__ uint16_t f2bf_bits(float f) { return __builtin_bit_cast(uint16_t, f2bf(f)); }
__device__ __forceinline__ float bf_bits2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Corner vertices and trilinear weights (FP64) of the data-grid cell holding the
// position p in [-1, 1]^3: c = (p + 1)/2 (n - 1) per axis, clamped to [0, n - 1]
// (NaN to 0), base = min(floor(c), n - 2), f = c - base.
// Every operation is a correctly rounded IEEE double operation in a fixed order
// (no contraction), so the weights are reproducible bit for bit.
__device__ __forceinline__ void data_cell(const float *p, int nx, int ny, int nz, int64_t v[8],
                                          double w[8]) {
#pragma clang fp contract(off)
    const int n[3] = {nx, ny, nz};
    int64_t b[3];
    double f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double c = ((double)p[a] + 1.0) * 0.5 * (double)(n[a] - 1);
        c = c == c ? fmin(fmax(c, 0.0), (double)(n[a] - 1)) : 0.0;
        const int bb = min((int)c, n[a] - 2);
        b[a] = bb;
        f[a] = c - (double)bb;
    }
#pragma unroll
    for (int cn = 0; cn < 8; ++cn) {
        const int dx = cn & 1, dy = (cn >> 1) & 1, dz = (cn >> 2) & 1;
        v[cn] = (b[0] + dx) + (int64_t)nx * ((b[1] + dy) + (int64_t)ny * (b[2] + dz));
        w[cn] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
    }
}

// Copies the host list ref_v[n_ref] of reference vertices into device memory dst
// through kernel arguments (64 per launch) instead of a pageable host copy, which
// would make the host wait for the stream; stream-ordered like any launch.
int put_refs(const int64_t *ref_v, int n_ref, int64_t *dst, hipStream_t st);

// Bytes at the start of a workspace that hold the int32 device status word
// (NDF_OK, or NDF_E_NONFINITE once a call has met a non-finite input or loss).
constexpr size_t kStatusBytes = 256;
int launch_status_clear(int32_t *status, hipStream_t st);

inline int status_of_launch() { return hipGetLastError() == hipSuccess ? NDF_OK : NDF_E_HIP; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

}  // namespace ndf
