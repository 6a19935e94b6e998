// Direct Pearson dependence fields (Sec. 3.1, Eq. 1).
//
// With per-vertex population mean mu_v and 1/sigma_v from ndf_prepare,
//   r(ref, v) = (1/N) sum_m z_ref[m] * (x[m][v] - mu_v) * inv_std_v,
//   z_ref[m]  = (x[m][ref] - mu_ref) * inv_std_ref.
// The ensemble is member-major, so a member row is a contiguous stream over
// vertices and every kernel below reads it with coalesced row segments.
//
// * pearson_gemv_kernel: one reference, FP32 FMA, four vertices per thread
//   (16-byte loads); bound by the 4 B/sample HBM stream.
// * pearson_gemm_kernel: up to 64 references at once as a contraction over
//   members on MFMA 32x32x16 bf16.  Standardised members are split into
//   z = hi + lo (both bf16) in registers and the three products hi*hi, hi*lo,
//   lo*hi are accumulated in FP32 (the lo*lo term is below 2^-16 relative).
//   The reference operand is prepared once per call in MFMA operand order.
// * pearson_pairs_kernel: one wave per vertex pair (training targets), from the
//   vertex-major integer codes with exact int64 moment sums.
#include "common.hpp"

namespace ndf {

// z_ref rows in FP32, zero-padded to kpad members: ws layout float[n_ref][kpad].
__global__ void pearson_refcols_kernel(const float *__restrict__ x, const double *__restrict__ mean,
                                       const double *__restrict__ inv_std, int N, int64_t V,
                                       const int64_t *__restrict__ refs, int kpad,
                                       float *__restrict__ zr) {
    const int r = blockIdx.x;
    const int64_t v = refs[r];
    const double mu = mean[v], is = inv_std[v];
    for (int m = threadIdx.x; m < kpad; m += blockDim.x) {
        float z = 0.f;
        if (m < N) z = (float)(((double)x[(int64_t)m * V + v] - mu) * is);
        zr[(int64_t)r * kpad + m] = z;
    }
}

// ---------------------------------------------------------------- GEMV ----
template <bool VEC>
__global__ __launch_bounds__(256) void pearson_gemv_kernel(
    const float *__restrict__ x, const double *__restrict__ mean,
    const double *__restrict__ inv_std, int N, int64_t V, const float *__restrict__ zr,
    float *__restrict__ out) {
    const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (v >= V) return;
    float mu[4], sc[4], acc[4] = {0.f, 0.f, 0.f, 0.f};
    const float invN = 1.0f / (float)N;
    for (int e = 0; e < 4; ++e) {
        const int64_t ve = v + e < V ? v + e : V - 1;
        mu[e] = (float)mean[ve];
        sc[e] = (float)(inv_std[ve] / (double)N);
    }
    (void)invN;
    if (VEC) {
        const f32x4 *xp = reinterpret_cast<const f32x4 *>(x + v);
        const int64_t row = V / 4;
#pragma unroll 8
        for (int m = 0; m < N; ++m) {
            const f32x4 a = __builtin_nontemporal_load(xp + (int64_t)m * row);
            const float z = zr[m];
            acc[0] = fmaf(z, a[0] - mu[0], acc[0]);
            acc[1] = fmaf(z, a[1] - mu[1], acc[1]);
            acc[2] = fmaf(z, a[2] - mu[2], acc[2]);
            acc[3] = fmaf(z, a[3] - mu[3], acc[3]);
        }
    } else {
        for (int m = 0; m < N; ++m) {
            const float z = zr[m];
            for (int e = 0; e < 4; ++e)
                if (v + e < V) acc[e] = fmaf(z, x[(int64_t)m * V + v + e] - mu[e], acc[e]);
        }
    }
    for (int e = 0; e < 4; ++e)
        if (v + e < V) out[v + e] = acc[e] * sc[e];
}

// ---------------------------------------------------------------- GEMM ----
// A operand (references) in MFMA order, ws layout:
//   bf16 frag[ks][ib][part][lane][8], part 0 = hi, 1 = lo,
//   lane l holds ref ib*32 + l%32, members ks*16 + 8*(l/32) + e.
__global__ void pearson_afrag_kernel(const float *__restrict__ zr, int kpad, int n_ib,
                                     int n_ref, uint16_t *__restrict__ frag) {
    const int ks = blockIdx.x;
    const int ib = blockIdx.y;
    const int lane = threadIdx.x;  // 64
    const int r = ib * 32 + (lane & 31);
    for (int e = 0; e < 8; ++e) {
        const int m = ks * 16 + 8 * (lane >> 5) + e;
        const float z = (r < n_ref) ? zr[(int64_t)r * kpad + m] : 0.f;
        const uint16_t hi = f2bf_bits(z);
        const uint16_t lo = f2bf_bits(z - bf_bits2f(hi));
        const int64_t base = (((int64_t)ks * n_ib + ib) * 2) * 64 * 8;
        frag[base + lane * 8 + e] = hi;
        frag[base + 64 * 8 + lane * 8 + e] = lo;
    }
}

// z = (x - mu) * sigma^-1 split into bf16 hi + lo: hi is z rounded, lo the
// exact product minus hi (one FMA) rounded, so every kernel below splits an
// element into the same two values.
__device__ __forceinline__ void split_z(float x, float mu, float is, __bf16 &hi, __bf16 &lo) {
    const float d = x - mu;
    const __bf16 hb = f2bf(d * is);
    hi = hb;
    lo = f2bf(__builtin_fmaf(d, is, -(float)hb));
}

// Each wave computes NIB 32-ref blocks x 64 vertices.  Lane l loads the vertex
// pair 2 (l%32), 2 (l%32) + 1 of its member rows as one 8-byte access, so tile
// t (0, 1) column j is vertex v0 + 2 j + t: a 256-byte contiguous segment per
// member row and lane half.  The next k-step's loads are issued before the
// current one's MFMAs, and the per-wave register footprint is kept small
// enough for three waves per SIMD.  Skipped loads (past the last member or
// vertex) read as 0: the reference operand is zero past the last member and
// columns past the last vertex are never stored.
constexpr int kGemmVerts = 64;

template <int NIB, bool VEC>
__global__ __launch_bounds__(256) void pearson_gemm_kernel(
    const float *__restrict__ x, const double *__restrict__ mean,
    const double *__restrict__ inv_std, int N, int64_t V, const bf16x8 *__restrict__ afrag,
    int n_ib_total, int n_ref, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int jl = lane & 31;
    const int ib0 = blockIdx.y * NIB;  // first 32-ref block of this group
    const int64_t v0 = ((int64_t)blockIdx.x * 4 + wave) * kGemmVerts + 2 * jl;  // tile t: v0 + t

    float mu[2], is[2];
    bool ok[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        ok[t] = v0 + t < V;
        const int64_t vv = ok[t] ? v0 + t : 0;
        mu[t] = (float)mean[vv];
        is[t] = (float)inv_std[vv];
    }

    f32x16 acc[NIB][2];
#pragma unroll
    for (int i = 0; i < NIB; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][t][r] = 0.f;

    // raw member values of one k-step: xv[e][t] = x[m0 + e][v0 + t]
    auto load = [&](int ks, float (&xv)[8][2]) {
        const int m0 = ks * 16 + 8 * h;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int m = m0 + e;
            const float *row = x + (int64_t)(m < N ? m : 0) * V;
            if (VEC) {
                f32x2 a = {0.f, 0.f};
                if (m < N && ok[0]) a = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(row + v0));
                xv[e][0] = a[0];
                xv[e][1] = a[1];
            } else {
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    xv[e][t] = (m < N && ok[t]) ? __builtin_nontemporal_load(row + v0 + t) : 0.f;
            }
        }
    };

    const int ksteps = (N + 15) / 16;
    float cur[8][2], nxt[8][2];
    load(0, cur);
    for (int ks = 0; ks < ksteps; ++ks) {
        if (ks + 1 < ksteps) load(ks + 1, nxt);
        bf16x8 bhi[2], blo[2];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                __bf16 hb, lb;
                split_z(cur[e][t], mu[t], is[t], hb, lb);
                bhi[t][e] = hb;
                blo[t][e] = lb;
            }
#pragma unroll
        for (int i = 0; i < NIB; ++i) {
            const int64_t fb = (((int64_t)ks * n_ib_total + ib0 + i) * 2) * 64;
            const bf16x8 ahi = afrag[fb + lane];
            const bf16x8 alo = afrag[fb + 64 + lane];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                acc[i][t] = mfma32(ahi, bhi[t], acc[i][t]);
                acc[i][t] = mfma32(ahi, blo[t], acc[i][t]);
                acc[i][t] = mfma32(alo, bhi[t], acc[i][t]);
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            cur[e][0] = nxt[e][0];
            cur[e][1] = nxt[e][1];
        }
    }
    const float invN = 1.0f / (float)N;
#pragma unroll
    for (int i = 0; i < NIB; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ref = (ib0 + i) * 32 + d_row(r, lane);
            if (ref >= n_ref) continue;
            float *o = out + (int64_t)ref * V + v0;
            if (VEC && ok[0]) {
                f32x2 y = {acc[i][0][r] * invN, acc[i][1][r] * invN};
                *reinterpret_cast<f32x2 *>(o) = y;
            } else {
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (ok[t]) o[t] = acc[i][t][r] * invN;
            }
        }
}

// Many references in one read of the ensemble: a workgroup of four waves takes
// 128 vertices and 256 references, wave w the references 64 w .. 64 w + 63 for
// all 128 vertices (four 32-vertex tiles, 128 accumulators: the reference
// fragments, read from L2, are the per-MFMA traffic, so each is used for as
// many vertices as the registers allow).  Each k-step (16 members) the
// workgroup loads the 16 x 128 block of x once (one member row segment of 512
// bytes per 128 threads), standardises and splits it into hi/lo bf16 and
// stages it in LDS in MFMA B-operand order; all four waves read their B
// operands from there.  Three LDS buffers, one barrier per k-step: step ks
// multiplies on buffer ks % 3, stages x of step ks + 2 into buffer (ks + 2) % 3
// and loads x of step ks + 4 (two k-steps to arrive, three register sets); the
// B operands of tiles 0 and 1 are read a step ahead (during the previous step's
// MFMAs), those of tiles 2 and 3 at the start of the step, behind tiles 0 and
// 1's MFMAs, so no MFMA waits for an LDS read issued after the barrier.  No load
// sits behind a branch (rows past the last member read member N - 1, where the
// reference operand is zero, and columns past the last vertex read a real
// vertex): with a branch the compiler's wait for the fragments also drains the
// x loads just issued.  The per-element split and the order of the MFMAs per
// accumulator match pearson_gemm_kernel, so both give the same bits.
constexpr int kWideVerts = 128;
constexpr int kWideTiles = kWideVerts / 32;
constexpr int kWideRefs = 256;

__global__ __launch_bounds__(256, 2) void pearson_gemm_wide_kernel(
    const float *__restrict__ x, const double *__restrict__ mean,
    const double *__restrict__ inv_std, int N, int64_t V, const bf16x8 *__restrict__ afrag,
    int n_ib_total, int n_ref, float *__restrict__ out) {
    __shared__ bf16x8 s_bop[3][kWideTiles][2][64];  // [buffer][vertex tile][hi, lo][lane]
    const int tid = threadIdx.x;
    const int lane = tid & 63, jl = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t vbase = (int64_t)blockIdx.x * kWideVerts;
    const int ib0 = blockIdx.y * (kWideRefs / 32) + 2 * wave;  // this wave's two 32-ref blocks
    const bool active = ib0 * 32 < n_ref;
    // an idle wave (past the last reference) fetches real fragments it never uses
    const int ibf = min(ib0, n_ib_total - 2);

    // loader role: vertex vj of the block, members 8 mh .. 8 mh + 7 of the k-step;
    // the thread then owns one 16-byte B-operand slot per part, so the LDS writes
    // of a wave are conflict-free
    const int vj = tid & (kWideVerts - 1);
    const int mh = __builtin_amdgcn_readfirstlane(tid >> 7);  // uniform per wave
    const int64_t vg = vbase + vj;
    const int64_t vgc = vg < V ? vg : V - 1;
    const float mu = (float)mean[vgc], is = (float)inv_std[vgc];
    const float *col = x + vgc;
    auto load = [&](int ks, float (&xv)[8]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int m = min(ks * 16 + 8 * mh + e, N - 1);
            xv[e] = __builtin_nontemporal_load(col + (int64_t)m * V);
        }
    };
    // B operand element (member k, vertex j): tile j / 32, lane 32 (k / 8) + j % 32,
    // position k % 8
    auto stage = [&](const float (&xv)[8], int buf) {
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            __bf16 hb, lb;
            split_z(xv[e], mu, is, hb, lb);
            hi[e] = hb;
            lo[e] = lb;
        }
        const int t = vj >> 5, ln = 32 * mh + (vj & 31);
        s_bop[buf][t][0][ln] = hi;
        s_bop[buf][t][1][ln] = lo;
    };
    const int ksteps = (N + 15) / 16;
    auto afetch = [&](int ks, bf16x8 (&a)[2][2]) {
        const int kc = min(ks, ksteps - 1);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t fb = (((int64_t)kc * n_ib_total + ibf + i) * 2) * 64;
            a[i][0] = afrag[fb + lane];
            a[i][1] = afrag[fb + 64 + lane];
        }
    };
    // tiles 0 and 1 of a step's B operands (hi, lo), read a step ahead
    auto bfetch01 = [&](int buf, bf16x8 (&bp)[2][2]) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            bp[t][0] = s_bop[buf][t][0][lane];
            bp[t][1] = s_bop[buf][t][1][lane];
        }
    };

    f32x16 acc[2][kWideTiles];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < kWideTiles; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][t][r] = 0.f;

    // step ks: MFMAs on buffer ks % 3 (tiles 0, 1 from registers read a step
    // earlier, tiles 2, 3 read now), tiles 0, 1 of step ks + 1 read ahead, x of
    // step ks + 2 staged into buffer (ks + 2) % 3 (last read in step ks - 1, before
    // the previous barrier) and x of step ks + 4 loaded
    auto step = [&](int ks, const bf16x8 (&acur)[2][2], bf16x8 (&anext)[2][2],
                    const bf16x8 (&bcur)[2][2], bf16x8 (&bnext)[2][2],
                    const float (&xstage)[8], float (&xload)[8]) {
        const int buf = ks % 3;
        afetch(ks + 1, anext);
        if (active) {
            bf16x8 b23[2][2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                b23[t][0] = s_bop[buf][2 + t][0][lane];
                b23[t][1] = s_bop[buf][2 + t][1][lane];
            }
            // the same per-accumulator order as the other kernels: hi.hi, hi.lo, lo.hi
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][t] = mfma32(acur[i][0], bcur[t][0], acc[i][t]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][t] = mfma32(acur[i][0], bcur[t][1], acc[i][t]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][t] = mfma32(acur[i][1], bcur[t][0], acc[i][t]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][2 + t] = mfma32(acur[i][0], b23[t][0], acc[i][2 + t]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][2 + t] = mfma32(acur[i][0], b23[t][1], acc[i][2 + t]);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 2; ++i) acc[i][2 + t] = mfma32(acur[i][1], b23[t][0], acc[i][2 + t]);
            bfetch01((ks + 1) % 3, bnext);
        }
        stage(xstage, (ks + 2) % 3);
        load(ks + 4, xload);
        __syncthreads();
    };
    float x0[8], x1[8], x2[8];
    bf16x8 a0[2][2], a1[2][2], b0[2][2], b1[2][2];
    afetch(0, a0);
    load(0, x0);
    load(1, x1);
    load(2, x2);
    stage(x0, 0);
    stage(x1, 1);
    load(3, x0);
    __syncthreads();
    if (active) bfetch01(0, b0);
    // x(j) lives in set j % 3 of {x0, x1, x2}: step ks stages x(ks + 2) and loads
    // x(ks + 4) into the set that x(ks + 1) left in the step before
    int ks = 0;
    for (; ks + 5 < ksteps; ks += 6) {
        step(ks, a0, a1, b0, b1, x2, x1);
        step(ks + 1, a1, a0, b1, b0, x0, x2);
        step(ks + 2, a0, a1, b0, b1, x1, x0);
        step(ks + 3, a1, a0, b1, b0, x2, x1);
        step(ks + 4, a0, a1, b0, b1, x0, x2);
        step(ks + 5, a1, a0, b1, b0, x1, x0);
    }
    if (ks < ksteps) step(ks, a0, a1, b0, b1, x2, x1);
    if (ks + 1 < ksteps) step(ks + 1, a1, a0, b1, b0, x0, x2);
    if (ks + 2 < ksteps) step(ks + 2, a0, a1, b0, b1, x1, x0);
    if (ks + 3 < ksteps) step(ks + 3, a1, a0, b1, b0, x2, x1);
    if (ks + 4 < ksteps) step(ks + 4, a0, a1, b0, b1, x0, x2);
    if (!active) return;
    const float invN = 1.0f / (float)N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ref = (ib0 + i) * 32 + d_row(r, lane);
            if (ref >= n_ref) continue;
#pragma unroll
            for (int t = 0; t < kWideTiles; ++t) {
                const int64_t v = vbase + 32 * t + jl;
                if (v < V) out[(int64_t)ref * V + v] = acc[i][t][r] * invN;
            }
        }
}

// --------------------------------------------------------------- pairs ----
// Training targets for random vertex pairs.  A pair's two member columns are
// strided rows of the member-major ensemble (one 128-byte line per value), so
// the pairs path reads the vertex-major integer codes instead: one contiguous
// row of N codes per vertex.  Pearson's r is invariant to the per-vertex affine
// map that defines the codes; their rounding to 2^-23 of the vertex range moves
// r by well under 1e-6.  The five moment sums are exact in int64 (codes < 2^24,
// N <= 4096), and r follows from them in FP64.
__device__ __forceinline__ long long wave_sum_i64(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <bool VEC>
__global__ __launch_bounds__(256) void pearson_pairs_kernel(
    const int32_t *__restrict__ code_a, const int32_t *__restrict__ code_b,
    const int32_t *__restrict__ flags_a, const int32_t *__restrict__ flags_b, int N, int64_t V,
    const int64_t *__restrict__ pairs, int64_t B, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;
    const int64_t va = pairs[2 * b], vb = pairs[2 * b + 1];
    if (va < 0 || va >= V || vb < 0 || vb >= V) {
        if (lane == 0) out[b] = __builtin_nanf("");
        return;
    }
    const int32_t f = flags_a[va] | flags_b[vb];
    if (f & (NDF_FLAG_NONFINITE | NDF_FLAG_CONSTANT)) {
        if (lane == 0) out[b] = (f & NDF_FLAG_NONFINITE) ? __builtin_nanf("") : 0.0f;
        return;
    }
    const int32_t *ra = code_a + va * N, *rb = code_b + vb * N;
    long long sa = 0, sb = 0, saa = 0, sbb = 0, sab = 0;
    auto add = [&](int x, int y) {
        sa += x;
        sb += y;
        saa += (long long)x * x;
        sbb += (long long)y * y;
        sab += (long long)x * y;
    };
    if (VEC) {  // N % 4 == 0: 16-byte rows
        for (int m = 4 * lane; m < N; m += 256) {
            const i32x4 x = *reinterpret_cast<const i32x4 *>(ra + m);
            const i32x4 y = *reinterpret_cast<const i32x4 *>(rb + m);
#pragma unroll
            for (int e = 0; e < 4; ++e) add(x[e], y[e]);
        }
    } else {
        for (int m = lane; m < N; m += 64) add(ra[m], rb[m]);
    }
    sa = wave_sum_i64(sa);
    sb = wave_sum_i64(sb);
    saa = wave_sum_i64(saa);
    sbb = wave_sum_i64(sbb);
    sab = wave_sum_i64(sab);
    if (lane == 0) {
        const double n = (double)N, da = (double)sa, db = (double)sb;
        const double cov = (double)sab - da * db / n;
        const double var_a = (double)saa - da * da / n;
        const double var_b = (double)sbb - db * db / n;
        out[b] = (float)(cov / sqrt(var_a * var_b));
    }
}

// --------------------------------------------------- continuous positions ----
// Pearson's r between the interpolated local samples at two positions (targets
// at continuous positions): one wave per pair; the sixteen corner columns are
// rows of the vertex-major copy xt (coalesced).  Member m's centred sample is
// sum_c w_c (x_m(v_c) - mean(v_c)) in FP64; corners of weight 0 are skipped (a
// non-finite value there does not reach the result).
template <bool VEC>
__global__ __launch_bounds__(256) void pearson_points_kernel(
    const float *__restrict__ xt_a, const float *__restrict__ xt_b,
    const double *__restrict__ mean_a, const double *__restrict__ mean_b,
    const int32_t *__restrict__ flags_a, const int32_t *__restrict__ flags_b, int N, int nx,
    int ny, int nz, const float *__restrict__ pos, int64_t B, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;
    int64_t va[8], vb[8];
    double wa[8], wb[8];
    data_cell(pos + 6 * b, nx, ny, nz, va, wa);
    data_cell(pos + 6 * b + 3, nx, ny, nz, vb, wb);
    bool bad = false;
    double mua[8], mub[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        bad |= wa[c] != 0.0 && (flags_a[va[c]] & NDF_FLAG_NONFINITE);
        bad |= wb[c] != 0.0 && (flags_b[vb[c]] & NDF_FLAG_NONFINITE);
        mua[c] = mean_a[va[c]];
        mub[c] = mean_b[vb[c]];
    }
    if (bad) {
        if (lane == 0) out[b] = __builtin_nanf("");
        return;
    }
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    if (VEC) {  // N % 4 == 0: 16-byte loads of every corner row
        for (int m = 4 * lane; m < N; m += 256) {
            f32x4 xa[8], xb[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                xa[c] = *reinterpret_cast<const f32x4 *>(xt_a + va[c] * N + m);
                xb[c] = *reinterpret_cast<const f32x4 *>(xt_b + vb[c] * N + m);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                double da = 0.0, db = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (wa[c] != 0.0) da += wa[c] * ((double)xa[c][e] - mua[c]);
                    if (wb[c] != 0.0) db += wb[c] * ((double)xb[c][e] - mub[c]);
                }
                sab += da * db;
                saa += da * da;
                sbb += db * db;
            }
        }
    } else {
        for (int m = lane; m < N; m += 64) {
            double da = 0.0, db = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (wa[c] != 0.0) da += wa[c] * ((double)xt_a[va[c] * N + m] - mua[c]);
                if (wb[c] != 0.0) db += wb[c] * ((double)xt_b[vb[c] * N + m] - mub[c]);
            }
            sab += da * db;
            saa += da * da;
            sbb += db * db;
        }
    }
    sab = wave_sum_f64(sab);
    saa = wave_sum_f64(saa);
    sbb = wave_sum_f64(sbb);
    if (lane == 0) out[b] = (saa > 0.0 && sbb > 0.0) ? (float)(sab / sqrt(saa * sbb)) : 0.0f;
}

// ------------------------------------------------------------ launchers ----
size_t pearson_ws_bytes(int N, int n_ref, int prec) {
    const int kpad = (int)align_up((size_t)N, 16);
    size_t zr = align_up((size_t)n_ref * kpad * sizeof(float), 256);
    size_t refs = align_up((size_t)n_ref * sizeof(int64_t), 256);
    if (prec == NDF_PREC_SPLIT_BF16) {
        const int n_ib = (int)ceil_div(n_ref, 64) * 2;
        size_t frag = (size_t)(kpad / 16) * n_ib * 2 * 64 * 8 * sizeof(uint16_t);
        return zr + refs + align_up(frag, 256);
    }
    return zr + refs;
}

int launch_pearson_field(const ndf_ensemble *e, int var_ref, int var_qry, const int64_t *ref_v,
                         int n_ref, float *out, int prec, void *ws, hipStream_t st) {
    const int N = e->n_members;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    const int kpad = (int)align_up((size_t)N, 16);
    char *w = (char *)ws;
    float *zr = (float *)w;
    w += align_up((size_t)n_ref * kpad * sizeof(float), 256);
    int64_t *refs = (int64_t *)w;
    w += align_up((size_t)n_ref * sizeof(int64_t), 256);
    if (put_refs(ref_v, n_ref, refs, st) != NDF_OK) return NDF_E_HIP;
    const float *xr = e->x + (int64_t)var_ref * N * V;
    const float *xq = e->x + (int64_t)var_qry * N * V;
    hipLaunchKernelGGL(pearson_refcols_kernel, dim3(n_ref), dim3(256), 0, st, xr,
                       e->mean + (int64_t)var_ref * V, e->inv_std + (int64_t)var_ref * V, N, V,
                       refs, kpad, zr);
    const double *mq = e->mean + (int64_t)var_qry * V;
    const double *iq = e->inv_std + (int64_t)var_qry * V;
    if (prec == NDF_PREC_FP32) {
        const unsigned nb = (unsigned)ceil_div(ceil_div(V, 4), 256);
        const bool vec = (V % 4) == 0;
        for (int r = 0; r < n_ref; ++r) {
            if (vec)
                hipLaunchKernelGGL(pearson_gemv_kernel<true>, dim3(nb), dim3(256), 0, st, xq, mq,
                                   iq, N, V, zr + (int64_t)r * kpad, out + (int64_t)r * V);
            else
                hipLaunchKernelGGL(pearson_gemv_kernel<false>, dim3(nb), dim3(256), 0, st, xq, mq,
                                   iq, N, V, zr + (int64_t)r * kpad, out + (int64_t)r * V);
        }
        return status_of_launch();
    }
    // split-bf16 MFMA contraction, references in groups of 64 (or one 32-block)
    const int n_ib = (int)ceil_div(n_ref, 64) * 2;
    uint16_t *frag = (uint16_t *)w;
    hipLaunchKernelGGL(pearson_afrag_kernel, dim3(kpad / 16, n_ib), dim3(64), 0, st, zr, kpad,
                       n_ib, n_ref, frag);
    const unsigned nbx = (unsigned)ceil_div(V, 4 * kGemmVerts);
    // 8-byte accesses need every member row 8-byte aligned: V even
    const bool vec = (V % 2) == 0;
    const bf16x8 *af = (const bf16x8 *)frag;
    if (n_ref > 64) {
        // one read of the ensemble per 256 references
        const dim3 g((unsigned)ceil_div(V, kWideVerts), (unsigned)ceil_div(n_ref, kWideRefs));
        hipLaunchKernelGGL(pearson_gemm_wide_kernel, g, dim3(256), 0, st, xq, mq, iq, N, V, af,
                           n_ib, n_ref, out);
    } else if (n_ref <= 32) {
        const dim3 g(nbx, 1);
        if (vec)
            hipLaunchKernelGGL((pearson_gemm_kernel<1, true>), g, dim3(256), 0, st, xq, mq, iq, N,
                               V, af, n_ib, n_ref, out);
        else
            hipLaunchKernelGGL((pearson_gemm_kernel<1, false>), g, dim3(256), 0, st, xq, mq, iq, N,
                               V, af, n_ib, n_ref, out);
    } else {
        const dim3 g(nbx, (unsigned)ceil_div(n_ref, 64));
        if (vec)
            hipLaunchKernelGGL((pearson_gemm_kernel<2, true>), g, dim3(256), 0, st, xq, mq, iq, N,
                               V, af, n_ib, n_ref, out);
        else
            hipLaunchKernelGGL((pearson_gemm_kernel<2, false>), g, dim3(256), 0, st, xq, mq, iq, N,
                               V, af, n_ib, n_ref, out);
    }
    return status_of_launch();
}

int launch_pearson_pairs(const ndf_ensemble *e, int var_a, int var_b, const int64_t *pairs,
                         int64_t B, float *out, hipStream_t st) {
    const int N = e->n_members;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    const int32_t *ca = e->code + (int64_t)var_a * V * N;
    const int32_t *cb = e->code + (int64_t)var_b * V * N;
    const int32_t *fa = e->flags + (int64_t)var_a * V;
    const int32_t *fb = e->flags + (int64_t)var_b * V;
    const dim3 g((unsigned)ceil_div(B, 4));
    if (N % 4 == 0)
        hipLaunchKernelGGL(pearson_pairs_kernel<true>, g, dim3(256), 0, st, ca, cb, fa, fb, N, V,
                           pairs, B, out);
    else
        hipLaunchKernelGGL(pearson_pairs_kernel<false>, g, dim3(256), 0, st, ca, cb, fa, fb, N, V,
                           pairs, B, out);
    return status_of_launch();
}

int launch_pearson_points(const ndf_ensemble *e, int var_a, int var_b, const float *pos,
                          int64_t B, float *out, hipStream_t st) {
    const int N = e->n_members;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    const float *xa = e->xt + (int64_t)var_a * V * N;
    const float *xb = e->xt + (int64_t)var_b * V * N;
    const double *ma = e->mean + (int64_t)var_a * V, *mb = e->mean + (int64_t)var_b * V;
    const int32_t *fa = e->flags + (int64_t)var_a * V, *fb = e->flags + (int64_t)var_b * V;
    const dim3 g((unsigned)ceil_div(B, 4));
    if (N % 4 == 0)
        hipLaunchKernelGGL(pearson_points_kernel<true>, g, dim3(256), 0, st, xa, xb, ma, mb, fa, fb,
                           N, e->nx, e->ny, e->nz, pos, B, out);
    else
        hipLaunchKernelGGL(pearson_points_kernel<false>, g, dim3(256), 0, st, xa, xb, ma, mb, fa,
                           fb, N, e->nx, e->ny, e->nz, pos, B, out);
    return status_of_launch();
}

}  // namespace ndf
