// Host-side description of the learned-field network (Sec. 4.1-4.2): config
// checks, the FP32 parameter layout and the workspace plans of the network calls.
#pragma once

#include "common.hpp"

namespace ndf {

constexpr int kH = 128;      // hidden width
constexpr int kF = 8;        // features per grid level
constexpr int kL = 4;        // grid levels
constexpr int kK0 = kL * kF; // encoder input width (grid features)
// With Fourier features (Sec. 4.2, Eq. 4): kFourierL frequencies; the encoder input
// is the 32 grid features, the raw position (3) and 6 kFourierL sines and cosines,
// zero-padded to kK0F = 112 (7 k-blocks of the MFMA).
constexpr int kFourierL = 12;
constexpr int kK0F = 112;

inline int enc_in(const ndf_net_config *c) { return c->fourier ? kK0F : kK0; }
constexpr int64_t kAlign = 64;

struct NetOffsets {
    int64_t grid[2][kL];
    int64_t W1[2], b1[2], W2[2], b2[2], W3[2], b3[2];
    int64_t W4, b4, W5, b5, w6, b6;
    int64_t cells[kL];
    int64_t total;  // floats
};

inline int check_net_config(const ndf_net_config *c) {
    if (!c) return NDF_E_ARG;
    if (c->nx < 2 || c->ny < 2 || c->nz < 2) return NDF_E_ARG;
    // the trilinear lookup divides exactly by multiply-high: numerators below
    // 2^24 (vertex indices, i (R - 1)), divisors below 2^16
    if (c->nx > 65535 || c->ny > 65535 || c->nz > 65535) return NDF_E_UNSUPPORTED;
    if ((int64_t)c->nx * c->ny * c->nz >= (1 << 24)) return NDF_E_UNSUPPORTED;
    if (c->n_levels != kL || c->feats != kF || c->width != kH) return NDF_E_UNSUPPORTED;
    if (c->n_enc != 1 && c->n_enc != 2) return NDF_E_ARG;
    if (c->grid_only != 0 && c->grid_only != 1) return NDF_E_ARG;
    if (c->fourier != 0 && c->fourier != kFourierL) return NDF_E_ARG;
    // Fourier features feed the encoder MLP of a shared-encoder network
    if (c->fourier && (c->n_enc != 1 || c->grid_only)) return NDF_E_UNSUPPORTED;
    for (int l = 0; l < kL; ++l)
        for (int a = 0; a < 3; ++a)
            if (c->res[l][a] < 2 || c->res[l][a] > (1 << 16)) return NDF_E_ARG;
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int l = 0; l < kL; ++l)
        for (int a = 0; a < 3; ++a)
            if ((int64_t)(n[a] - 1) * (c->res[l][a] - 1) >= (1 << 24)) return NDF_E_UNSUPPORTED;
    // hash tables of 2^T entries (T = log2_hashmap, 0: every level dense)
    const int T = c->log2_hashmap;
    if (T != 0 && (T < 8 || T > 24)) return NDF_E_ARG;
    for (int l = 0; l < kL; ++l) {
        const int64_t dense = (int64_t)c->res[l][0] * c->res[l][1] * c->res[l][2];
        const bool hashed = T != 0 && dense > ((int64_t)1 << T);
        if (!hashed && dense >= ((int64_t)1 << 28)) return NDF_E_UNSUPPORTED;  // int32 cell offsets
    }
    return NDF_OK;
}

// Level l is stored as a hash table of 2^T entries when its dense size exceeds
// that (the multi-resolution hash grid of Sec. 4.2), else densely.
inline bool level_hashed(const ndf_net_config *c, int l) {
    const int64_t dense = (int64_t)c->res[l][0] * c->res[l][1] * c->res[l][2];
    return c->log2_hashmap != 0 && dense > ((int64_t)1 << c->log2_hashmap);
}

inline NetOffsets net_offsets(const ndf_net_config *c) {
    NetOffsets o{};
    int64_t pos = 0;
    auto take = [&](int64_t n) {
        int64_t at = pos;
        pos += (n + kAlign - 1) / kAlign * kAlign;
        return at;
    };
    for (int l = 0; l < kL; ++l)
        o.cells[l] = level_hashed(c, l) ? ((int64_t)1 << c->log2_hashmap)
                                        : (int64_t)c->res[l][0] * c->res[l][1] * c->res[l][2];
    for (int e = 0; e < c->n_enc; ++e) {
        for (int l = 0; l < kL; ++l) o.grid[e][l] = take(o.cells[l] * kF);
        if (c->grid_only) continue;  // no encoder MLP (W1..b3 offsets stay 0, unused)
        o.W1[e] = take(kH * enc_in(c));
        o.b1[e] = take(kH);
        o.W2[e] = take(kH * kH);
        o.b2[e] = take(kH);
        o.W3[e] = take(kH * kH);
        o.b3[e] = take(kH);
    }
    if (c->n_enc == 1) {
        for (int l = 0; l < kL; ++l) o.grid[1][l] = o.grid[0][l];
        o.W1[1] = o.W1[0]; o.b1[1] = o.b1[0];
        o.W2[1] = o.W2[0]; o.b2[1] = o.b2[0];
        o.W3[1] = o.W3[0]; o.b3[1] = o.b3[0];
    }
    o.W4 = take(kH * (c->grid_only ? kK0 : kH));
    o.b4 = take(kH);
    o.W5 = take(kH * kH);
    o.b5 = take(kH);
    o.w6 = take(kH);
    o.b6 = take(1);
    o.total = pos;
    return o;
}

// Level geometry passed by value to kernels.
struct GridGeom {
    int nx, ny, nz;
    int R[kL][3];
    float inv[3];        // 1 / (n - 1) per axis
    uint64_t md[3];      // ceil(2^40 / (n - 1)) per axis
    uint64_t mx, my;     // ceil(2^40 / nx), ceil(2^40 / ny)
    uint32_t hmask[kL];  // table entries - 1 for a hashed level, 0 for a dense one
};

inline GridGeom grid_geom(const ndf_net_config *c) {
    GridGeom g{};
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    for (int l = 0; l < kL; ++l)
        for (int a = 0; a < 3; ++a) g.R[l][a] = c->res[l][a];
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        g.inv[a] = 1.0f / (float)(n[a] - 1);
        g.md[a] = ((1ull << 40) + (uint64_t)(n[a] - 2)) / (uint64_t)(n[a] - 1);
    }
    g.mx = ((1ull << 40) + (uint64_t)c->nx - 1) / (uint64_t)c->nx;
    g.my = ((1ull << 40) + (uint64_t)c->ny - 1) / (uint64_t)c->ny;
    for (int l = 0; l < kL; ++l)
        g.hmask[l] = level_hashed(c, l) ? (uint32_t)((1u << c->log2_hashmap) - 1) : 0u;
    return g;
}

// Cell of level corner (x, y, z): dense x + Rx (y + Ry z), or on a hashed level
// (hm = table entries - 1) the spatial hash of the hash grids that Sec. 4.2
// builds on (Mueller et al. 2022): (x * 1 xor y * 2654435761 xor z * 805459861)
// mod 2^T in 32-bit unsigned arithmetic.  HASH = false compiles the dense form
// only (every level dense).
template <bool HASH>
__device__ __forceinline__ int cell_index(int x, int y, int z, const int R[3], uint32_t hm) {
    const uint32_t dense = (uint32_t)x + (uint32_t)R[0] * ((uint32_t)y + (uint32_t)R[1] * (uint32_t)z);
    if (!HASH) return (int)dense;
    const uint32_t h = (uint32_t)x ^ ((uint32_t)y * 2654435761u) ^ ((uint32_t)z * 805459861u);
    return (int)(hm ? (h & hm) : dense);
}

__device__ __forceinline__ uint32_t level_hmask(const GridGeom &g, int l) {
    return l == 0 ? g.hmask[0] : (l == 1 ? g.hmask[1] : (l == 2 ? g.hmask[2] : g.hmask[3]));
}

// Level sizes of level l (l may differ between lanes: selects instead of an
// indexed load keep the geometry in scalar registers).
__device__ __forceinline__ void level_dims(const GridGeom &g, int l, int R[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
        R[a] = l == 0 ? g.R[0][a] : (l == 1 ? g.R[1][a] : (l == 2 ? g.R[2][a] : g.R[3][a]));
}

// Trilinear corners of grid vertex v on a level of sizes R: cell indices and
// weights.  c = u (R - 1) with u = i / (n - 1), evaluated as one correctly
// rounded division i (R - 1) / (n - 1) (exact whenever c is an integer);
// base = clamp(floor(c), 0, R - 2), f = c - base; corner (dx,dy,dz) = bit 0,1,2.
// Vertex and cell indices fit in 32 bits (V, cells < 2^31).
template <bool HASH = false>
__device__ __forceinline__ void corners_R32(const GridGeom &g, const int R[3], int64_t v64,
                                            int idx[8], float w[8], uint32_t hm = 0) {
    const uint32_t v = (uint32_t)v64;
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    // exact divisions by multiply-high: numerators < 2^24, divisors < 2^16
    const uint32_t t = (uint32_t)(((uint64_t)v * g.mx) >> 40);  // v / nx
    const uint32_t k = (uint32_t)(((uint64_t)t * g.my) >> 40);  // t / ny
    const uint32_t ii[3] = {v - t * nx, t - k * ny, k};
    const int nn[3] = {g.nx, g.ny, g.nz};
    int b[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // c = i (R - 1) / (n - 1) = q + rem / (n - 1): cell q (at most R - 2), so a
        // vertex on a level vertex gets weight exactly 1 and its neighbour 0
        const uint32_t p = ii[a] * (uint32_t)(R[a] - 1);
        const uint32_t q = (uint32_t)(((uint64_t)p * g.md[a]) >> 40);
        const uint32_t rem = p - q * (uint32_t)(nn[a] - 1);
        const int bb = min((int)q, R[a] - 2);
        b[a] = bb;
        f[a] = (float)((int)q - bb) + (float)rem * g.inv[a];
    }
#pragma unroll
    for (int cn = 0; cn < 8; ++cn) {
        const int dx = cn & 1, dy = (cn >> 1) & 1, dz = (cn >> 2) & 1;
        idx[cn] = cell_index<HASH>(b[0] + dx, b[1] + dy, b[2] + dz, R, hm);
        w[cn] = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) * (dz ? f[2] : 1.f - f[2]);
    }
}

// Trilinear corners of a continuous position p in the network's input domain
// [-1, 1]^3 (Sec. 4.3) on a level of sizes R: c = (p + 1)/2 (R - 1) per axis as one
// FP32 fma, clamped to [0, R - 1], so positions outside the domain (and NaN, which
// the max turns into 0) take the boundary's value; base = min(floor(c), R - 2),
// f = c - base.  The position 2 i/(n - 1) - 1 of vertex i gives the vertex lookup's
// cell, with weights equal up to the rounding of c.
template <bool HASH = false>
__device__ __forceinline__ void corners_pos32(const int R[3], const float p[3], int idx[8],
                                              float w[8], uint32_t hm = 0) {
    int b[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hr = 0.5f * (float)(R[a] - 1);
        const float c = fminf(fmaxf(fmaf(p[a], hr, hr), 0.f), (float)(R[a] - 1));
        const int bb = min(max((int)c, 0), R[a] - 2);
        b[a] = bb;
        f[a] = c - (float)bb;
    }
#pragma unroll
    for (int cn = 0; cn < 8; ++cn) {
        const int dx = cn & 1, dy = (cn >> 1) & 1, dz = (cn >> 2) & 1;
        idx[cn] = cell_index<HASH>(b[0] + dx, b[1] + dy, b[2] + dz, R, hm);
        w[cn] = (dx ? f[0] : 1.f - f[0]) * (dy ? f[1] : 1.f - f[1]) * (dz ? f[2] : 1.f - f[2]);
    }
}

// ------------------------------------------- packed bf16 helpers (MFMA epilogues) ----
typedef __attribute__((ext_vector_type(2))) short s16x2;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// Two floats -> packed bf16 pair (a in the low half), round to nearest even.  A
// two-element vector conversion maps to the two-source v_cvt_pk_bf16_f32; the
// scalar form would convert each value on its own and merge the halves.  (No
// inline asm here: the compiler does not see an asm statement's reads of MFMA
// results and would not insert the wait states they need.)
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// ReLU of a packed bf16 pair: a bf16 is negative iff its sign bit is set, so a
// signed 16-bit max with 0 (one v_pk_max_i16) clamps both halves.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
    const s16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), z));
}
// max(x, 0) as a signed integer max on the bit pattern: negative floats have
// the sign bit set, so they compare below 0 and map to +0.  (fmaxf would first
// quiet NaNs with an extra max per value.)
__device__ __forceinline__ float relu_f32(float x) {
    return __int_as_float(max(__float_as_int(x), 0));
}
__device__ __forceinline__ float bf_lo(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float bf_hi(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }

// --------------------------------------------------- Fourier features ----
// Position p in [-1, 1]^3 of grid vertex v: p_a = (2 i_a - (n_a - 1)) / (n_a - 1)
// (one rounding), the vertex decomposed as in corners_R32.
__device__ __forceinline__ void vertex_p(const GridGeom &g, int64_t v64, float p[3]) {
    const uint32_t v = (uint32_t)v64;
    const uint32_t t = (uint32_t)(((uint64_t)v * g.mx) >> 40);  // v / nx
    const uint32_t k = (uint32_t)(((uint64_t)t * g.my) >> 40);  // t / ny
    const int ii[3] = {(int)(v - t * (uint32_t)g.nx), (int)(t - k * (uint32_t)g.ny), (int)k};
    const int nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = (float)(2 * ii[a] - (nn[a] - 1)) / (float)(nn[a] - 1);
}
// A continuous position clamped to the domain (NaN -> -1), as the lookup clamps it.
__device__ __forceinline__ void clamp_p(const float q[3], float p[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf(q[a], -1.f), 1.f);
}

__host__ __device__ constexpr float pow2f(int n) {
    return n >= 0 ? (float)(1u << n) : 1.f / (float)(1u << -n);
}
// Slot t of the 80 inputs after the grid features: the raw position (t < 3),
// sin and cos of 2^i pi p_j (t = 3 + 6 i + 2 j, + 1 for cos), zero padding
// (t >= 75).  sin(2^i pi p) is the hardware sine of x = 2^(i-1) p revolutions
// reduced exactly to x - rint(x) in [-1/2, 1/2]; cos adds a quarter turn.
__device__ __forceinline__ float ff_value(int t, const float (&p)[3]) {
    if (t < 3) return p[t];
    if (t >= 3 + 6 * kFourierL) return 0.f;
    const int u = t - 3;
    const float x = p[(u % 6) / 2] * pow2f(u / 6 - 1);
    return __builtin_amdgcn_sinf(x - rintf(x) + ((u & 1) ? 0.25f : 0.f));
}
// Element e of k-block kb >= 2 of the encoder input, lane half h: slot
// t = 16 (kb - 2) + 8 h + e.  Both halves' slots are known at compile time, so
// the lane picks its argument first and evaluates one sine.
__device__ __forceinline__ float ff_elem(int kb, int e, int h, const float (&p)[3]) {
    const int t0 = 16 * (kb - 2) + e, t1 = t0 + 8;
    const bool f0 = t0 >= 3 && t0 < 3 + 6 * kFourierL, f1 = t1 >= 3 && t1 < 3 + 6 * kFourierL;
    if (f0 && f1) {
        const int u0 = t0 - 3, u1 = t1 - 3;
        const float x = h ? p[(u1 % 6) / 2] * pow2f(u1 / 6 - 1) : p[(u0 % 6) / 2] * pow2f(u0 / 6 - 1);
        const float q = h ? ((u1 & 1) ? 0.25f : 0.f) : ((u0 & 1) ? 0.25f : 0.f);
        return __builtin_amdgcn_sinf(x - rintf(x) + q);
    }
    const float v0 = ff_value(t0, p), v1 = ff_value(t1, p);
    return h ? v1 : v0;
}
__device__ __forceinline__ bf16x8 ff_chunk(int kb, int h, const float (&p)[3]) {
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = f2bf(ff_elem(kb, e, h, p));
    return r;
}

size_t net_train_ws_bytes(const ndf_net_config *c, int64_t B);
size_t net_infer_ws_bytes(const ndf_net_config *c, int64_t n_ref, int prec);
size_t net_infer_lat_ws_bytes(int64_t n_ref);
size_t net_qparam_bytes(const ndf_net_config *c, int prec);

int launch_net_init(const ndf_net_config *c, float *params, float *opt, uint64_t seed,
                    hipStream_t st);
// Rows come from vertex pairs int64[B][2] (pos null) or from continuous
// position pairs float[B][2][3] in [-1, 1]^3 (pairs null).
int launch_net_grad(const ndf_net_config *c, const float *params, const int64_t *pairs,
                    const float *pos, const float *targets, int64_t B, float *grad, float *loss,
                    void *ws, hipStream_t st);
int launch_net_forward(const ndf_net_config *c, const float *params, const int64_t *pairs,
                       const float *pos, int64_t B, float *y, void *ws, hipStream_t st);
int launch_adam(const ndf_net_config *c, float *params, float *opt, const float *grad,
                int64_t step, float lr, const int32_t *status, hipStream_t st);
int launch_net_quantize(const ndf_net_config *c, const float *params, int prec, void *q,
                        hipStream_t st);
int launch_net_swap_encoders(const ndf_net_config *c, const float *in, float *out,
                             hipStream_t st);
size_t net_latent_cache_bytes(const ndf_net_config *c);
int launch_infer_latents(const ndf_net_config *c, const void *q, void *cache, hipStream_t st);
int launch_infer_field_cached(const ndf_net_config *c, const void *q, const int64_t *ref_v,
                              int n_ref, const void *cache, float *out, void *ws, hipStream_t st);
int launch_infer_field(const ndf_net_config *c, const void *q, int prec, const int64_t *ref_v,
                       int n_ref, float *out, void *ws, hipStream_t st);
int launch_infer_points(const ndf_net_config *c, const void *q, int prec, const int64_t *ref_v,
                        int n_ref, const float *pos, int64_t n, float *out, void *ws,
                        hipStream_t st);
int launch_infer_difference(const ndf_net_config *c, const void *q, int64_t ref_a, int64_t ref_b,
                            const void *cache, float *out, void *ws, hipStream_t st);

}  // namespace ndf
