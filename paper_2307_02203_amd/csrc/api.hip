// extern "C" entry points of libndf.so: host-side validation, workspace carving
// and dispatch to the kernel launchers.  Nothing here allocates, frees or
// synchronises; every call enqueues on the caller's stream.
#include <math.h>
#include <string.h>

#include <mutex>

#include "common.hpp"
#include "net.hpp"

namespace ndf {
int launch_prepare(const ndf_ensemble *e, int32_t *status, hipStream_t st);
size_t pearson_ws_bytes(int N, int n_ref, int prec);
int launch_pearson_field(const ndf_ensemble *e, int var_ref, int var_qry, const int64_t *ref_v,
                         int n_ref, float *out, int prec, void *ws, hipStream_t st);
int launch_pearson_pairs(const ndf_ensemble *e, int var_a, int var_b, const int64_t *pairs,
                         int64_t B, float *out, hipStream_t st);
int launch_pearson_points(const ndf_ensemble *e, int var_a, int var_b, const float *pos,
                          int64_t B, float *out, hipStream_t st);
size_t ksg_field_ws_bytes(int N, int n_ref);
int launch_ksg_field(const ndf_ensemble *e, int var_ref, int var_qry, const int64_t *ref_v,
                     int n_ref, int k, float *out, int32_t *counts, void *ws, hipStream_t st);
size_t ksg_pairs_ws_bytes(int N);
int launch_ksg_orders(const ndf_ensemble *e, hipStream_t st);
int launch_ksg_pairs(const ndf_ensemble *e, int var_a, int var_b, const int64_t *pairs, int64_t B,
                     int k, float *out, int32_t *counts, double *H, hipStream_t st);
size_t ksg_points_ws_bytes(int N, int64_t B);
int launch_ksg_points(const ndf_ensemble *e, int var_a, int var_b, const float *pos, int64_t B,
                      int k, float *out, int32_t *counts, void *ws, hipStream_t st);
}  // namespace ndf

using namespace ndf;

// ------------------------------------------- field without allocation ----
// Device scratch of the no-allocation KSG field call: the workspace of
// launch_ksg_field (harmonic table, reference list, sorted reference columns)
// for requests up to kKsgScratchBytes.  Every device holds its own copy for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is not a device
// address in host code).  Calls on one device share the array, so calls that
// overlap in time on one device race; each call writes every byte it reads.
namespace {

constexpr size_t kKsgScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kKsgScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // per device, set once by the first call there

int ksg_scratch_ptr(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NDF_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NDF_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NDF_OK;
}

}  // namespace

namespace {

constexpr int kMaxMembers = 4096;
constexpr int kMaxMembersKsg = 2048;

int64_t n_vertices(const ndf_ensemble *e) { return (int64_t)e->nx * e->ny * e->nz; }

int check_ensemble(const ndf_ensemble *e, bool need_stats) {
    if (!e || !e->x) return NDF_E_ARG;
    if (e->n_members < 2 || e->n_members > kMaxMembers) return NDF_E_ARG;
    if (e->nx < 2 || e->ny < 2 || e->nz < 2 || e->n_vars < 1) return NDF_E_ARG;
    if (need_stats && (!e->mean || !e->inv_std || !e->code || !e->flags)) return NDF_E_ARG;
    return NDF_OK;
}

int check_var(const ndf_ensemble *e, int v) { return (v >= 0 && v < e->n_vars) ? NDF_OK : NDF_E_ARG; }

int check_refs(const ndf_ensemble *e, const int64_t *ref_v, int n_ref) {
    if (!ref_v || n_ref < 1) return NDF_E_ARG;
    const int64_t V = n_vertices(e);
    for (int r = 0; r < n_ref; ++r)
        if (ref_v[r] < 0 || ref_v[r] >= V) return NDF_E_ARG;
    return NDF_OK;
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

namespace ndf {

struct RefBatch {
    int64_t v[64];
};

__global__ void put_refs_kernel(RefBatch rb, int n, int64_t *__restrict__ dst) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = rb.v[threadIdx.x];
}

int put_refs(const int64_t *ref_v, int n_ref, int64_t *dst, hipStream_t st) {
    for (int r0 = 0; r0 < n_ref; r0 += 64) {
        RefBatch rb{};
        const int n = n_ref - r0 < 64 ? n_ref - r0 : 64;
        for (int i = 0; i < n; ++i) rb.v[i] = ref_v[r0 + i];
        hipLaunchKernelGGL(put_refs_kernel, dim3(1), dim3(64), 0, st, rb, n, dst + r0);
    }
    return status_of_launch();
}

}  // namespace ndf

extern "C" {

const char *ndf_status_string(int s) {
    switch (s) {
        case NDF_OK: return "ok";
        case NDF_E_ARG: return "invalid argument";
        case NDF_E_WORKSPACE: return "workspace missing or too small";
        case NDF_E_HIP: return "HIP launch failed";
        case NDF_E_UNSUPPORTED: return "unsupported configuration";
        case NDF_E_NONFINITE: return "non-finite value (input or loss)";
        case NDF_E_SCRATCH: return "request exceeds the library's static device scratch";
        default: return "unknown status";
    }
}

size_t ndf_workspace_bytes(int32_t op, const ndf_ensemble *ens, const ndf_net_config *net,
                           int64_t n, int32_t prec) {
    switch (op) {
        case NDF_OP_PEARSON_FIELD:
            if (check_ensemble(ens, false) != NDF_OK || n < 1 || n > (1 << 20)) return 0;
            if (prec != NDF_PREC_FP32 && prec != NDF_PREC_SPLIT_BF16) return 0;
            return pearson_ws_bytes(ens->n_members, (int)n, prec);
        case NDF_OP_KSG_FIELD:
            if (check_ensemble(ens, false) != NDF_OK || n < 1 || n > (1 << 20)) return 0;
            return ksg_field_ws_bytes(ens->n_members, (int)n);
        case NDF_OP_KSG_PAIRS:
            if (check_ensemble(ens, false) != NDF_OK) return 0;
            return ksg_pairs_ws_bytes(ens->n_members);
        case NDF_OP_KSG_POINTS:
            if (check_ensemble(ens, false) != NDF_OK || n < 1 || n > (1ll << 29)) return 0;
            return ksg_points_ws_bytes(ens->n_members, n);
        case NDF_OP_TRAIN:
            if (check_net_config(net) != NDF_OK || n < 1) return 0;
            return net_train_ws_bytes(net, n);
        case NDF_OP_PREPARE:
            return check_ensemble(ens, false) == NDF_OK ? kStatusBytes : 0;
        case NDF_OP_INFER:
            if (check_net_config(net) != NDF_OK || n < 1 || n > (1 << 20)) return 0;
            return net_infer_ws_bytes(net, n, prec);
        case NDF_OP_INFER_CACHED:
            if (check_net_config(net) != NDF_OK || n < 1 || n > (1 << 20)) return 0;
            return net_infer_lat_ws_bytes(n);
        default: return 0;
    }
}

int ndf_prepare(const ndf_ensemble *ens, void *ws, size_t ws_bytes, void *stream) {
    int s = check_ensemble(ens, true);
    if (s != NDF_OK) return s;
    if (ws && ws_bytes < kStatusBytes) return NDF_E_WORKSPACE;
    s = launch_prepare(ens, (int32_t *)ws, S(stream));
    if (s == NDF_OK && ens->order) s = launch_ksg_orders(ens, S(stream));
    return s;
}

int ndf_pearson_field(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                      const int64_t *ref_v, int32_t n_ref, float *out, int32_t prec, void *ws,
                      size_t ws_bytes, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_ref);
    if (s == NDF_OK) s = check_var(ens, var_qry);
    if (s == NDF_OK) s = check_refs(ens, ref_v, n_ref);
    if (s != NDF_OK) return s;
    if (!out) return NDF_E_ARG;
    if (prec != NDF_PREC_FP32 && prec != NDF_PREC_SPLIT_BF16) return NDF_E_UNSUPPORTED;
    if (!ws || ws_bytes < pearson_ws_bytes(ens->n_members, n_ref, prec)) return NDF_E_WORKSPACE;
    return launch_pearson_field(ens, var_ref, var_qry, ref_v, n_ref, out, prec, ws, S(stream));
}

int ndf_ksg_mi_field(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                     const int64_t *ref_v, int32_t n_ref, int32_t k, float *out,
                     int32_t *counts, void *ws, size_t ws_bytes, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_ref);
    if (s == NDF_OK) s = check_var(ens, var_qry);
    if (s == NDF_OK) s = check_refs(ens, ref_v, n_ref);
    if (s != NDF_OK) return s;
    if (!out || k < 1 || k >= ens->n_members) return NDF_E_ARG;
    if (k > 8 || ens->n_members > kMaxMembersKsg) return NDF_E_UNSUPPORTED;
    if (!ws || ws_bytes < ksg_field_ws_bytes(ens->n_members, n_ref)) return NDF_E_WORKSPACE;
    return launch_ksg_field(ens, var_ref, var_qry, ref_v, n_ref, k, out, counts, ws, S(stream));
}

size_t ndf_ksg_scratch_bytes(void) { return kKsgScratchBytes; }

int ndf_ksg_mi_field_noalloc(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                             const int64_t *ref_v, int32_t n_ref, int32_t k, float *out,
                             int32_t *counts, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_ref);
    if (s == NDF_OK) s = check_var(ens, var_qry);
    if (s == NDF_OK) s = check_refs(ens, ref_v, n_ref);
    if (s != NDF_OK) return s;
    if (!out || k < 1 || k >= ens->n_members) return NDF_E_ARG;
    if (k > 8 || ens->n_members > kMaxMembersKsg) return NDF_E_UNSUPPORTED;
    if (n_ref > (1 << 20) || ksg_field_ws_bytes(ens->n_members, n_ref) > kKsgScratchBytes)
        return NDF_E_SCRATCH;
    void *ws = nullptr;
    s = ksg_scratch_ptr(&ws);
    if (s != NDF_OK) return s;
    return launch_ksg_field(ens, var_ref, var_qry, ref_v, n_ref, k, out, counts, ws, S(stream));
}

int ndf_pearson_pairs(const ndf_ensemble *ens, int32_t var_a, int32_t var_b,
                      const int64_t *pairs, int64_t B, float *out, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_a);
    if (s == NDF_OK) s = check_var(ens, var_b);
    if (s != NDF_OK) return s;
    if (!pairs || !out || B < 1) return NDF_E_ARG;
    return launch_pearson_pairs(ens, var_a, var_b, pairs, B, out, S(stream));
}

int ndf_pearson_points(const ndf_ensemble *ens, int32_t var_a, int32_t var_b, const float *pos,
                       int64_t B, float *out, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_a);
    if (s == NDF_OK) s = check_var(ens, var_b);
    if (s != NDF_OK) return s;
    if (!ens->xt || B < 0 || (B > 0 && (!pos || !out))) return NDF_E_ARG;
    if (B == 0) return NDF_OK;
    return launch_pearson_points(ens, var_a, var_b, pos, B, out, S(stream));
}

int ndf_ksg_mi_pairs(const ndf_ensemble *ens, int32_t var_a, int32_t var_b,
                     const int64_t *pairs, int64_t B, int32_t k, float *out, int32_t *counts,
                     void *ws, size_t ws_bytes, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_a);
    if (s == NDF_OK) s = check_var(ens, var_b);
    if (s != NDF_OK) return s;
    if (!pairs || !out || B < 1 || k < 1 || k >= ens->n_members) return NDF_E_ARG;
    if (k > 8 || ens->n_members > kMaxMembersKsg) return NDF_E_UNSUPPORTED;
    if (!ws || ws_bytes < ksg_pairs_ws_bytes(ens->n_members)) return NDF_E_WORKSPACE;
    return launch_ksg_pairs(ens, var_a, var_b, pairs, B, k, out, counts, (double *)ws, S(stream));
}

int ndf_ksg_mi_points(const ndf_ensemble *ens, int32_t var_a, int32_t var_b, const float *pos,
                      int64_t B, int32_t k, float *out, int32_t *counts, void *ws,
                      size_t ws_bytes, void *stream) {
    int s = check_ensemble(ens, true);
    if (s == NDF_OK) s = check_var(ens, var_a);
    if (s == NDF_OK) s = check_var(ens, var_b);
    if (s != NDF_OK) return s;
    if (!ens->xt || B < 0 || B > (1ll << 29) || (B > 0 && (!pos || !out)) || k < 1 ||
        k >= ens->n_members)
        return NDF_E_ARG;
    if (k > 8 || ens->n_members > kMaxMembersKsg) return NDF_E_UNSUPPORTED;
    if (B == 0) return NDF_OK;
    if (!ws || ws_bytes < ksg_points_ws_bytes(ens->n_members, B)) return NDF_E_WORKSPACE;
    return launch_ksg_points(ens, var_a, var_b, pos, B, k, out, counts, ws, S(stream));
}

size_t ndf_net_param_bytes(const ndf_net_config *cfg) {
    if (check_net_config(cfg) != NDF_OK) return 0;
    return (size_t)net_offsets(cfg).total * sizeof(float);
}

size_t ndf_net_optstate_bytes(const ndf_net_config *cfg) { return 2 * ndf_net_param_bytes(cfg); }

int ndf_net_init(const ndf_net_config *cfg, float *params, float *opt_state, uint64_t seed,
                 void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params) return NDF_E_ARG;
    return launch_net_init(cfg, params, opt_state, seed, S(stream));
}

int ndf_net_grad(const ndf_net_config *cfg, const float *params, const int64_t *pairs,
                 const float *targets, int64_t B, float *grad_out, float *loss_out, void *ws,
                 size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !pairs || !targets || !grad_out || !loss_out || B < 1) return NDF_E_ARG;
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B)) return NDF_E_WORKSPACE;
    return launch_net_grad(cfg, params, pairs, nullptr, targets, B, grad_out, loss_out, ws,
                           S(stream));
}

int ndf_net_grad_at(const ndf_net_config *cfg, const float *params, const float *pos,
                    const float *targets, int64_t B, float *grad_out, float *loss_out, void *ws,
                    size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !pos || !targets || !grad_out || !loss_out || B < 1) return NDF_E_ARG;
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B)) return NDF_E_WORKSPACE;
    return launch_net_grad(cfg, params, nullptr, pos, targets, B, grad_out, loss_out, ws,
                           S(stream));
}

int ndf_net_forward(const ndf_net_config *cfg, const float *params, const int64_t *pairs,
                    int64_t B, float *y, void *ws, size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !pairs || !y || B < 1) return NDF_E_ARG;
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B)) return NDF_E_WORKSPACE;
    return launch_net_forward(cfg, params, pairs, nullptr, B, y, ws, S(stream));
}

int ndf_net_forward_at(const ndf_net_config *cfg, const float *params, const float *pos,
                       int64_t B, float *y, void *ws, size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !pos || !y || B < 1) return NDF_E_ARG;
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B)) return NDF_E_WORKSPACE;
    return launch_net_forward(cfg, params, nullptr, pos, B, y, ws, S(stream));
}

int ndf_train_step(const ndf_net_config *cfg, float *params, float *opt_state, int64_t step,
                   const int64_t *pairs, const float *targets, int64_t B, float lr,
                   float *loss_out, void *ws, size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !opt_state || !pairs || !targets || !loss_out || B < 1 || step < 1 ||
        !(lr >= 0.f) || !isfinite(lr))
        return NDF_E_ARG;
    const size_t pbytes = (size_t)net_offsets(cfg).total * sizeof(float);
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B) + align_up(pbytes, 256))
        return NDF_E_WORKSPACE;
    float *grad = (float *)((char *)ws + net_train_ws_bytes(cfg, B));
    s = launch_net_grad(cfg, params, pairs, nullptr, targets, B, grad, loss_out, ws, S(stream));
    if (s != NDF_OK) return s;
    return launch_adam(cfg, params, opt_state, grad, step, lr, (const int32_t *)ws, S(stream));
}

int ndf_train_step_at(const ndf_net_config *cfg, float *params, float *opt_state, int64_t step,
                      const float *pos, const float *targets, int64_t B, float lr,
                      float *loss_out, void *ws, size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !opt_state || !pos || !targets || !loss_out || B < 1 || step < 1 ||
        !(lr >= 0.f) || !isfinite(lr))
        return NDF_E_ARG;
    const size_t pbytes = (size_t)net_offsets(cfg).total * sizeof(float);
    if (!ws || ws_bytes < net_train_ws_bytes(cfg, B) + align_up(pbytes, 256))
        return NDF_E_WORKSPACE;
    float *grad = (float *)((char *)ws + net_train_ws_bytes(cfg, B));
    s = launch_net_grad(cfg, params, nullptr, pos, targets, B, grad, loss_out, ws, S(stream));
    if (s != NDF_OK) return s;
    return launch_adam(cfg, params, opt_state, grad, step, lr, (const int32_t *)ws, S(stream));
}

size_t ndf_net_qparam_bytes(const ndf_net_config *cfg, int32_t prec) {
    if (check_net_config(cfg) != NDF_OK) return 0;
    if (prec != NDF_PREC_BF16 && prec != NDF_PREC_FP8_E4M3) return 0;
    return net_qparam_bytes(cfg, prec);
}

int ndf_net_swap_encoders(const ndf_net_config *cfg, const float *params, float *params_out,
                          void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (cfg->n_enc != 2 || !params || !params_out || params == params_out) return NDF_E_ARG;
    return launch_net_swap_encoders(cfg, params, params_out, S(stream));
}

int ndf_net_quantize(const ndf_net_config *cfg, const float *params, int32_t prec, void *qparams,
                     void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!params || !qparams) return NDF_E_ARG;
    if (prec != NDF_PREC_BF16 && prec != NDF_PREC_FP8_E4M3) return NDF_E_UNSUPPORTED;
    if (cfg->grid_only && prec != NDF_PREC_BF16) return NDF_E_UNSUPPORTED;
    return launch_net_quantize(cfg, params, prec, qparams, S(stream));
}

int ndf_infer_field(const ndf_net_config *cfg, const void *qparams, int32_t prec,
                    const int64_t *ref_v, int32_t n_ref, float *out, void *ws, size_t ws_bytes,
                    void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!qparams || !out || !ref_v || n_ref < 1) return NDF_E_ARG;
    if (prec != NDF_PREC_BF16 && prec != NDF_PREC_FP8_E4M3) return NDF_E_UNSUPPORTED;
    if (cfg->grid_only && prec != NDF_PREC_BF16) return NDF_E_UNSUPPORTED;
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    for (int r = 0; r < n_ref; ++r)
        if (ref_v[r] < 0 || ref_v[r] >= V) return NDF_E_ARG;
    if (!ws || ws_bytes < net_infer_ws_bytes(cfg, n_ref, prec)) return NDF_E_WORKSPACE;
    return launch_infer_field(cfg, qparams, prec, ref_v, n_ref, out, ws, S(stream));
}

size_t ndf_infer_latent_bytes(const ndf_net_config *cfg) {
    return check_net_config(cfg) == NDF_OK ? net_latent_cache_bytes(cfg) : 0;
}

int ndf_infer_latents(const ndf_net_config *cfg, const void *qparams, void *cache, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!qparams || !cache) return NDF_E_ARG;
    if (cfg->grid_only) return NDF_E_UNSUPPORTED;
    return launch_infer_latents(cfg, qparams, cache, S(stream));
}

int ndf_infer_field_cached(const ndf_net_config *cfg, const void *qparams, const int64_t *ref_v,
                           int32_t n_ref, const void *cache, float *out, void *ws,
                           size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!qparams || !cache || !out || !ref_v || n_ref < 1) return NDF_E_ARG;
    if (cfg->grid_only) return NDF_E_UNSUPPORTED;
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    for (int r = 0; r < n_ref; ++r)
        if (ref_v[r] < 0 || ref_v[r] >= V) return NDF_E_ARG;
    if (!ws || ws_bytes < net_infer_lat_ws_bytes(n_ref)) return NDF_E_WORKSPACE;
    return launch_infer_field_cached(cfg, qparams, ref_v, n_ref, cache, out, ws, S(stream));
}

int ndf_infer_points(const ndf_net_config *cfg, const void *qparams, int32_t prec,
                     const int64_t *ref_v, int32_t n_ref, const float *pos, int64_t n, float *out,
                     void *ws, size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!qparams || !ref_v || n_ref < 1 || n < 0 || (n > 0 && (!pos || !out))) return NDF_E_ARG;
    if (prec != NDF_PREC_BF16 && prec != NDF_PREC_FP8_E4M3) return NDF_E_UNSUPPORTED;
    if (cfg->grid_only && prec != NDF_PREC_BF16) return NDF_E_UNSUPPORTED;
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    for (int r = 0; r < n_ref; ++r)
        if (ref_v[r] < 0 || ref_v[r] >= V) return NDF_E_ARG;
    if (!ws || ws_bytes < net_infer_ws_bytes(cfg, n_ref, prec)) return NDF_E_WORKSPACE;
    if (n == 0) return NDF_OK;
    return launch_infer_points(cfg, qparams, prec, ref_v, n_ref, pos, n, out, ws, S(stream));
}

int ndf_infer_field_difference(const ndf_net_config *cfg, const void *qparams, int64_t ref_a,
                               int64_t ref_b, const void *cache, float *out, void *ws,
                               size_t ws_bytes, void *stream) {
    int s = check_net_config(cfg);
    if (s != NDF_OK) return s;
    if (!qparams || !cache || !out) return NDF_E_ARG;
    if (cfg->grid_only) return NDF_E_UNSUPPORTED;
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    if (ref_a < 0 || ref_a >= V || ref_b < 0 || ref_b >= V) return NDF_E_ARG;
    if (!ws || ws_bytes < net_infer_lat_ws_bytes(2)) return NDF_E_WORKSPACE;
    return launch_infer_difference(cfg, qparams, ref_a, ref_b, cache, out, ws, S(stream));
}

}  // extern "C"
