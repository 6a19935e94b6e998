/*
 * ndf.h - C ABI of the MI355X (gfx950) hot path of neural dependence fields.
 *
 * Problem (Sec. 3): an ensemble of N members, each a scalar field per variable on
 * an nx*ny*nz grid.  For a reference vertex p_ref the dependence field
 * R(p_ref, .) holds, at every vertex p, a bivariate dependence measure between
 * the local samples e(p_ref) and e(p) (the N member values at those vertices):
 * Pearson's r (Sec. 3.1, Eq. 1) or mutual information by the nearest-neighbour
 * estimator of Kraskov et al. (Sec. 3.2, Eq. 2).  The learned field (Sec. 4,
 * Eq. 3) approximates R by a network Phi(p1, p2) that is trained on direct
 * estimates and evaluated at every vertex (Sec. 5).
 *
 * Conventions for every call
 *  - Pointers are DEVICE pointers unless marked [host].  The caller owns all
 *    memory, including the workspace `ws`; the library allocates, frees and
 *    synchronises nothing and keeps no pointer after a call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    only enqueue work on it; results are valid once the stream has reached
 *    that point.
 *  - Arguments are validated on the host before anything is enqueued: an
 *    invalid call returns a negative NDF_E_* status and enqueues nothing.
 *    NDF_E_HIP means a launch failed (hipGetLastError after the launch).
 *  - Vertex index v = i + nx*(j + ny*k); V = nx*ny*nz.
 *  - Calls that share a workspace must not overlap in time.
 *  - Device-side conditions cannot be returned by a call that only enqueues, so
 *    the calls that can meet them (ndf_prepare, the training calls) keep a
 *    device status word: the int32 at the start of their workspace `ws`.  The
 *    call resets it to NDF_OK first (a kernel, not a memset) and its kernels set
 *    it to NDF_E_NONFINITE when they meet a non-finite input value or loss; read
 *    it after the stream has passed the call.
 *
 * Build: libndf.so (hipcc --offload-arch=gfx950).  No function needs a GPU to be
 * looked up; every compute call needs one to run.
 */
#ifndef NDF_H
#define NDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NDF_OK = 0,
    NDF_E_ARG = -1,          /* null pointer, index or size out of range          */
    NDF_E_WORKSPACE = -2,    /* ws NULL or ws_bytes below ndf_workspace_bytes()   */
    NDF_E_HIP = -3,          /* a kernel launch failed                            */
    NDF_E_NONFINITE = -4,    /* device status word only: a non-finite input value
                                (ndf_prepare) or training loss was met            */
    NDF_E_UNSUPPORTED = -5,  /* valid request outside what the kernels implement  */
    NDF_E_SCRATCH = -6       /* request larger than the static device scratch of
                                ndf_ksg_mi_field_noalloc                          */
};

enum {
    NDF_PREC_FP32 = 0,       /* FP32 FMA stream (direct Pearson)                  */
    NDF_PREC_SPLIT_BF16 = 1, /* hi+lo BF16 MFMA, FP32 accumulate (direct Pearson) */
    NDF_PREC_BF16 = 2,       /* BF16 MFMA network, FP32 accumulate                */
    NDF_PREC_FP8_E4M3 = 3    /* OCP E4M3 weights/activations, FP32 accumulate     */
};

enum {                       /* `op` of ndf_workspace_bytes                       */
    NDF_OP_PEARSON_FIELD = 1,
    NDF_OP_KSG_FIELD = 2,
    NDF_OP_TRAIN = 3,
    NDF_OP_INFER = 4,
    NDF_OP_KSG_PAIRS = 5,
    NDF_OP_KSG_POINTS = 6,
    NDF_OP_PREPARE = 7,
    NDF_OP_INFER_CACHED = 8  /* ndf_infer_field_cached, ndf_infer_field_difference */
};

enum {                       /* per-vertex flags written by ndf_prepare           */
    NDF_FLAG_NONFINITE = 1,  /* a member value is NaN or infinite                 */
    NDF_FLAG_CONSTANT = 2    /* all member values are equal (zero range)          */
};

/* The ensemble (Sec. 3: members E_i, variables nu, local samples e^nu(p)). */
typedef struct ndf_ensemble {
    int32_t n_members;       /* N, 2 <= N <= 4096 (KSG calls: N <= 2048)          */
    int32_t nx, ny, nz;      /* grid; each >= 2                                   */
    int32_t n_vars;          /* d >= 1                                            */
    const float *x;          /* [n_vars][N][V] float32, member-major (input)      */
    double *mean;            /* [n_vars][V] population mean      (ndf_prepare)    */
    double *inv_std;         /* [n_vars][V] 1/population std, 0 where std == 0    */
    int32_t *code;           /* [n_vars][V][N] KSG integer codes, vertex-major    */
    int32_t *flags;          /* [n_vars][V] NDF_FLAG_* bits                       */
    uint16_t *order;         /* [n_vars][V][N] members in ascending (code, member)
                                order per vertex (ndf_prepare), or NULL: the KSG
                                calls then sort every column they use            */
    float *xt;               /* [n_vars][V][N] vertex-major copy of x written by
                                ndf_prepare, or NULL; needed only by the calls at
                                continuous positions (ndf_pearson_points)         */
} ndf_ensemble;

/* The learned field (Sec. 4.1-4.2): per encoder a dense multi-resolution feature
 * grid (n_levels levels of feats features, trilinear lookup) and an MLP
 * L*F -> W -> W -> W (ReLU after the first two layers, linear latent); the two
 * latents are multiplied element-wise and a decoder W -> W -> W -> 1 (ReLU,
 * ReLU, linear) gives Phi.  n_enc = 1: one encoder and grid for both positions
 * (self field, Phi symmetric); n_enc = 2: encoder 0 for p1, encoder 1 for p2.
 * Grid vertex (i,j,k) is at u = (i/(nx-1), j/(ny-1), k/(nz-1)).  The kernels
 * implement n_levels = 4, feats = 8, width = 128.  Limits (NDF_E_UNSUPPORTED
 * beyond them): nx*ny*nz < 2^24, each of nx, ny, nz <= 65535, and
 * (n-1)*(R-1) < 2^24 for every axis and level (the lookup's exact integer
 * arithmetic); a dense level holds fewer than 2^28 cells.
 * Hash grids (Sec. 4.2): with log2_hashmap = T in [8, 24], a level whose dense
 * size Rx*Ry*Rz exceeds 2^T is stored as a table of 2^T cells indexed by the
 * spatial hash (x * 1 xor y * 2654435761 xor z * 805459861) mod 2^T of the
 * corner (x, y, z) (32-bit unsigned arithmetic; the hash of the grids the paper
 * builds on, Mueller et al. 2022); coarser levels stay dense.  Colliding
 * corners share a cell (their gradients add).  T = 0: every level dense.
 * Grid-only network (grid_only = 1; the TensoRF-like ablation of Sec. 6.3,
 * Fig. 6: the encoder MLP omitted, predictions from the input embedding alone):
 * the latent of a position is its L*F = 32 grid features, the merge multiplies
 * the two 32-vectors and the decoder's first layer W4 is W x (L*F).  The
 * training, forward and BF16 field calls support it (ndf_infer_field with one
 * fused pass per reference, ndf_infer_points); FP8 and the query-latent calls
 * return NDF_E_UNSUPPORTED.
 * Fourier features (fourier = 12; Sec. 4.2, Eq. 4): the encoder input is the 32
 * grid features, then the raw position p in [-1, 1]^3 (vertex (i,j,k): p = 2u - 1;
 * a continuous position clamped to the domain, NaN -> -1), then for i < 12 and
 * j = x, y, z the pair sin(2^i pi p_j), cos(2^i pi p_j), then 5 zeros: 112
 * inputs, W1 is W x 112.  Requires n_enc = 1 and grid_only = 0
 * (NDF_E_UNSUPPORTED otherwise); every call supports it. */
typedef struct ndf_net_config {
    int32_t nx, ny, nz;      /* data grid whose vertices are evaluated            */
    int32_t n_levels;        /* 4                                                 */
    int32_t res[4][3];       /* level sizes (Rx, Ry, Rz), each >= 2               */
    int32_t feats;           /* 8                                                 */
    int32_t width;           /* 128                                               */
    int32_t n_enc;           /* 1 or 2                                            */
    int32_t log2_hashmap;    /* 0 (dense levels) or T in [8, 24]: hash tables of
                                2^T cells for the levels larger than that        */
    int32_t grid_only;       /* 0: full network; 1: encoder MLP omitted          */
    int32_t fourier;         /* 0, or 12: Fourier features of the position       */
} ndf_net_config;

/* Human-readable name of a status code (static storage). */
const char *ndf_status_string(int status);

/* Workspace bytes for `op`.  `ens` is used by the PEARSON/KSG ops, `net` by
 * TRAIN/INFER; n = n_ref for the field ops, B (pairs per step) for TRAIN and
 * KSG_POINTS.
 * `prec` as the call will use it.  Returns 0 for an invalid request. */
size_t ndf_workspace_bytes(int32_t op, const ndf_ensemble *ens, const ndf_net_config *net,
                           int64_t n, int32_t prec);

/* Standardisation and KSG codes, one pass set per ensemble (Sec. 3.1 Eq. 1
 * needs per-vertex means and variances; Sec. 3.2 the KSG neighbour search).
 * Writes mean, inv_std (FP64, population moments), flags, and for every vertex
 * v and member m the code rne((x - lo_v) * 2^23 / (hi_v - lo_v)) with lo/hi
 * the column min/max, all in IEEE double (0 for a constant column).  When
 * ens->order is non-NULL it also writes each vertex's members sorted by code
 * (ties by member index): the sorted orders the KSG neighbour search walks,
 * built once per ensemble instead of once per (reference, query) pair.
 * ws (nullable): ndf_workspace_bytes(NDF_OP_PREPARE, ens, NULL, 0, 0) bytes;
 * its status word becomes NDF_E_NONFINITE when any member value is NaN or
 * infinite (those vertices carry NDF_FLAG_NONFINITE).  NULL: no status word. */
int ndf_prepare(const ndf_ensemble *ens, void *ws, size_t ws_bytes, void *stream);

/* Direct Pearson field (Sec. 3.1, Eq. 1; Table 1 "Pearson"):
 * out[r][v] = r(e^{var_ref}(ref_v[r]), e^{var_qry}(v)) for r < n_ref, v < V.
 * ref_v [host] int64[n_ref].  prec NDF_PREC_FP32 streams the ensemble once per
 * reference; NDF_PREC_SPLIT_BF16 runs all references as one MFMA contraction of
 * standardised members (z = zhi + zlo, products hi*hi + hi*lo + lo*hi, FP32
 * accumulate).  r = 0 where either vertex has zero variance.  Needs ndf_prepare. */
int ndf_pearson_field(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                      const int64_t *ref_v, int32_t n_ref, float *out, int32_t prec,
                      void *ws, size_t ws_bytes, void *stream);

/* Direct KSG mutual-information field in nats (Sec. 3.2, Eq. 2; estimator of
 * [KSG04], first algorithm; Table 1 "MI"):  for the samples (x_m, y_m) =
 * (code[ref][m], code[v][m]), eps_m = k-th smallest max-norm distance to the
 * other samples, nx_m / ny_m = number of other samples strictly closer than
 * eps_m in x / y, and
 *   out[r][v] = psi(k) + psi(N) - (1/N) sum_m [psi(nx_m + 1) + psi(ny_m + 1)].
 * Counts are exact integers; the sum is FP64.  0 where either vertex is
 * constant.  counts (nullable) int32[n_ref][V][2][N] receives nx, ny in member
 * order.  1 <= k <= 8, k < N.  Needs ndf_prepare. */
int ndf_ksg_mi_field(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                     const int64_t *ref_v, int32_t n_ref, int32_t k, float *out,
                     int32_t *counts, void *ws, size_t ws_bytes, void *stream);

/* ndf_ksg_mi_field without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * ndf_ksg_mi_field (bit for bit); the workspace lives in a static device array
 * of ndf_ksg_scratch_bytes() bytes (1 MiB) that the library holds on every
 * device it runs on until the process ends.  The call allocates nothing; its
 * first call on a device looks up that device's scratch address (no
 * allocation).  Requests whose workspace, ndf_workspace_bytes(NDF_OP_KSG_FIELD,
 * ens, NULL, n_ref, 0), exceeds the scratch return NDF_E_SCRATCH with nothing
 * enqueued (at N = 1000 members up to 129 references per call; at N = 2048, 62).
 * All calls on one device share the scratch: calls that overlap in time on one
 * device (other streams, other host threads) race and must be serialised by the
 * caller.  Each call writes every scratch byte it reads, so stale contents of
 * an earlier call do not matter. */
size_t ndf_ksg_scratch_bytes(void);
int ndf_ksg_mi_field_noalloc(const ndf_ensemble *ens, int32_t var_ref, int32_t var_qry,
                             const int64_t *ref_v, int32_t n_ref, int32_t k, float *out,
                             int32_t *counts, void *stream);

/* Direct estimates for B vertex pairs (training targets of Eq. 3, Sec. 4.3):
 * out[b] = r or MI between e^{var_a}(pairs[b][0]) and e^{var_b}(pairs[b][1]),
 * with the definitions of ndf_pearson_field / ndf_ksg_mi_field.  pairs
 * int64[B][2] (device); a pair with an index outside [0, V) gives NaN.  Both
 * read the vertex-major codes of ndf_prepare (one contiguous row per vertex):
 * Pearson's r is invariant to the per-vertex affine map that defines a code,
 * and the rounding of the codes moves r by less than 1e-6.  KSG: counts
 * (nullable) int32[B][2][N] in member order; ws of
 * ndf_workspace_bytes(NDF_OP_KSG_PAIRS, ...) bytes. */
int ndf_pearson_pairs(const ndf_ensemble *ens, int32_t var_a, int32_t var_b,
                      const int64_t *pairs, int64_t B, float *out, void *stream);
int ndf_ksg_mi_pairs(const ndf_ensemble *ens, int32_t var_a, int32_t var_b,
                     const int64_t *pairs, int64_t B, int32_t k, float *out,
                     int32_t *counts, void *ws, size_t ws_bytes, void *stream);

/* Training targets at continuous positions (Sec. 4.3: pairs of positions drawn
 * from the domain, the ensemble sampled there by trilinear interpolation):
 * out[b] = r(e^{var_a}(p1), e^{var_b}(p2)) for pos float[B][2][3] (device;
 * p1 = pos[b][0], p2 = pos[b][1], x y z in [-1, 1]^3 with -1 and +1 the first
 * and last vertex of an axis, clamped to the domain).  The local sample at p is
 * e(p)_m = sum_c w_c x_m(v_c) over the eight vertices of the grid cell holding
 * p (data-grid coordinate c = (p + 1)/2 (n - 1), base = min(floor(c), n - 2),
 * trilinear weights), computed as sum_c w_c (x_m(v_c) - mean(v_c)) in FP64 so
 * the interpolated column is centred exactly; r from FP64 sums.  r = 0 where an
 * interpolated column has zero variance, NaN where a corner with nonzero weight
 * holds a non-finite value.  Reads ens->xt (NDF_E_ARG when NULL) and the means
 * of ndf_prepare.  B = 0 enqueues nothing. */
int ndf_pearson_points(const ndf_ensemble *ens, int32_t var_a, int32_t var_b, const float *pos,
                       int64_t B, float *out, void *stream);

/* KSG mutual information (nats) between the interpolated samples at position
 * pairs (Sec. 4.3 with the estimator of ndf_ksg_mi_field): each interpolated
 * column (the samples of ndf_pearson_points, summed over the corners of nonzero
 * weight in corner order in FP64, no contraction) is mapped to integer codes
 * exactly as ndf_prepare maps a vertex (min-max onto [0, 2^23], round-half-even),
 * so at a vertex's own position the codes, counts and estimate are that
 * vertex's.  out float[B]; counts (nullable) int32[B][2][N] in member order; 0
 * for a constant interpolated column, NaN for a non-finite one.  1 <= k <= 8,
 * k < N <= 2048, B <= 2^29.  ws: ndf_workspace_bytes(NDF_OP_KSG_POINTS, ens,
 * NULL, B, 0) bytes (the 2B code columns and their sorted member orders,
 * 12 B x N per pair, plus small tables).  Reads ens->xt (NDF_E_ARG when NULL).
 * B = 0 enqueues nothing. */
int ndf_ksg_mi_points(const ndf_ensemble *ens, int32_t var_a, int32_t var_b, const float *pos,
                      int64_t B, int32_t k, float *out, int32_t *counts, void *ws,
                      size_t ws_bytes, void *stream);

/* Bytes of the FP32 parameter vector (layout: for each encoder its grid levels
 * float[cells][feats] with cells = Rx*Ry*Rz, or 2^T for a hashed level, then
 * W1[W][L*F], b1, W2[W][W], b2, W3[W][W], b3 (absent for a grid-only network);
 * then W4[W][W] (grid-only: W4[W][L*F]), b4, W5[W][W], b5, w6[W], b6[1]; every
 * tensor starts at a multiple of 64 floats, gaps zero) and of the Adam state
 * (m then v, same layout). */
size_t ndf_net_param_bytes(const ndf_net_config *cfg);
size_t ndf_net_optstate_bytes(const ndf_net_config *cfg);

/* Seeded initialisation (He-uniform weights, zero biases, grid features
 * U(-1e-4, 1e-4)) from a counter-based generator (SplitMix64 of seed and
 * element index); also zeroes the Adam state when opt_state is non-NULL. */
int ndf_net_init(const ndf_net_config *cfg, float *params, float *opt_state, uint64_t seed,
                 void *stream);

/* Mean L1 loss over B pairs (Eq. 3 with d = L1, Sec. 4.3) and its gradient with
 * respect to every parameter (float[param_bytes/4], overwritten), by the
 * library's forward and adjoint kernels (BF16 MFMA, FP32 accumulate, FP32
 * atomic scatter into the grids).  pairs int64[B][2] (device), targets
 * float[B]; loss_out float[1] (device).  The workspace's status word becomes
 * NDF_E_NONFINITE when the loss is not finite (a NaN or infinite target or
 * output). */
int ndf_net_grad(const ndf_net_config *cfg, const float *params, const int64_t *pairs,
                 const float *targets, int64_t B, float *grad_out, float *loss_out,
                 void *ws, size_t ws_bytes, void *stream);

/* One training step of Eq. 3 (Sec. 4.3): ndf_net_grad followed by Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; `step` counts from 1).
 * opt_state holds m then v.  ws needs ndf_workspace_bytes(NDF_OP_TRAIN, .., B, ..)
 * plus the parameter bytes rounded up to 256; the gradient is left there.  A
 * step whose loss is not finite sets the status word to NDF_E_NONFINITE and
 * leaves params and opt_state unchanged (the Adam kernel reads the word). */
int ndf_train_step(const ndf_net_config *cfg, float *params, float *opt_state, int64_t step,
                   const int64_t *pairs, const float *targets, int64_t B, float lr,
                   float *loss_out, void *ws, size_t ws_bytes, void *stream);

/* The same three calls for pairs of continuous positions (Sec. 4.3 trains on
 * positions drawn from the domain, not only on grid vertices): pos float[B][2][3]
 * (device; pos[b][0] = p1, pos[b][1] = p2, x y z in [-1, 1]^3 with -1 and +1 the
 * first and last vertex of an axis; each grid level is interpolated trilinearly
 * at the position, coordinates outside the domain clamped, NaN to -1).  Targets
 * at such positions come from ndf_pearson_points.  Arguments and workspace
 * otherwise as for ndf_net_forward, ndf_net_grad and ndf_train_step. */
int ndf_net_forward_at(const ndf_net_config *cfg, const float *params, const float *pos,
                       int64_t B, float *y, void *ws, size_t ws_bytes, void *stream);
int ndf_net_grad_at(const ndf_net_config *cfg, const float *params, const float *pos,
                    const float *targets, int64_t B, float *grad_out, float *loss_out,
                    void *ws, size_t ws_bytes, void *stream);
int ndf_train_step_at(const ndf_net_config *cfg, float *params, float *opt_state, int64_t step,
                      const float *pos, const float *targets, int64_t B, float lr,
                      float *loss_out, void *ws, size_t ws_bytes, void *stream);

/* Multi-variable fields (Sec. 6.4): the network of the variable pair (nu, mu)
 * from that of (mu, nu), Phi_{nu mu}(p1, p2) = Phi_{mu nu}(p2, p1), by exchanging
 * the two encoders (grids and encoder layers); the decoder is shared.  With it,
 * d (d + 1) / 2 trained networks give all d^2 fields of a correlation volume
 * matrix.  cfg->n_enc must be 2.  params and params_out are FP32 parameter
 * blobs (ndf_net_param_bytes) in device memory that must not overlap.  Enqueues
 * one copy kernel.  Returns NDF_E_ARG for n_enc != 2, null or equal pointers. */
int ndf_net_swap_encoders(const ndf_net_config *cfg, const float *params, float *params_out,
                          void *stream);

/* Reduced-precision inference parameters (Sec. 5 evaluates the trained network
 * with 16-bit arithmetic): packed for `prec` (NDF_PREC_BF16 or
 * NDF_PREC_FP8_E4M3) from the FP32 parameters: BF16 grids, weights in MFMA
 * operand order, FP32 biases; FP8 adds E4M3 copies of layers 2..5 with E8M0
 * scales per output row and block of 32 inputs, and one static power-of-two
 * scale per layer input: the call runs the BF16 network on a fixed calibration
 * set (32 references x 2048 queries, vertex (2 i + 1) V / (2 n) for i < n) and
 * keeps M_l, the largest |input| of layer l = 2..5 (query-encoder activations,
 * latent product, first decoder activation); inference then scales layer l's
 * inputs by 2^-e_l, e_l the smallest exponent with 2 M_l <= 448 * 2^e_l, and
 * clamps them to +-448 * 2^e_l.  The four M_l (FP32 bits) are the first 16
 * bytes of the blob's last 256.  One packed blob serves both precisions
 * (grid-only networks: BF16 only, NDF_E_UNSUPPORTED for FP8). */
size_t ndf_net_qparam_bytes(const ndf_net_config *cfg, int32_t prec);
int ndf_net_quantize(const ndf_net_config *cfg, const float *params, int32_t prec,
                     void *qparams, void *stream);

/* Learned dependence field (Sec. 5): out[r][v] = Phi(p_ref[r], p_v) at every grid
 * vertex v, for ref_v [host] int64[n_ref] (out float[n_ref][V], device).  One
 * reference: every query is encoded, multiplied with the reference latent and
 * decoded in one fused kernel (grid gather + MFMA MLP), which also computes the
 * reference latent (once per workgroup, before its tiles; with two encoders from
 * encoder 0's layers), so a BF16 field is a single launch; FP8 with two encoders
 * computes the reference latents in a separate launch first.  BF16 with
 * n_ref >= 2: the query latents of all vertices are computed once into the
 * workspace (ndf_infer_latents) and every launch then decodes up to 16
 * references per read of them (ndf_infer_field_cached); the fields are the
 * single-reference fields bit for bit.  FP8 with n_ref = 1: layers 2..5 in E4M3
 * in one fused pass (two encoders: the reference latent first, in E4M3 too);
 * FP8 with n_ref >= 2: the query latents are cached in BF16 as above and only
 * the decoder (layers 4, 5) runs in E4M3, 16 references per read of the cache
 * (the BF16 network with an E4M3 decoder; its bar is that emulation's).
 * The call enqueues kernels only (no copies or memsets), so it can be captured
 * into a graph.  ws: ndf_workspace_bytes(NDF_OP_INFER, NULL, cfg, n_ref, prec)
 * bytes (n_ref >= 2: includes ndf_infer_latent_bytes(cfg) for the query
 * latents).  NDF_E_ARG for a null pointer, n_ref < 1 or a reference outside
 * [0, V). */
int ndf_infer_field(const ndf_net_config *cfg, const void *qparams, int32_t prec,
                    const int64_t *ref_v, int32_t n_ref, float *out, void *ws,
                    size_t ws_bytes, void *stream);

/* Many fields of one trained network (interactive exploration of references,
 * Sec. 5): the query latents e(p_v) do not depend on the reference, so they can
 * be computed once.  ndf_infer_latents writes the BF16 latents of the query
 * encoder for every grid vertex into `cache` (device, ndf_infer_latent_bytes
 * bytes, caller-owned; the fused kernel's register order, 256 bytes per
 * vertex); ndf_infer_field_cached then runs only the merge and the decoder per
 * reference, up to 16 references per launch, each launch reading every cached
 * latent once, and gives the same values as ndf_infer_field with NDF_PREC_BF16,
 * bit for bit.  ws: ndf_workspace_bytes(NDF_OP_INFER_CACHED, NULL, cfg, n_ref,
 * NDF_PREC_BF16) bytes (the reference latents). */
size_t ndf_infer_latent_bytes(const ndf_net_config *cfg);
int ndf_infer_latents(const ndf_net_config *cfg, const void *qparams, void *cache, void *stream);
int ndf_infer_field_cached(const ndf_net_config *cfg, const void *qparams, const int64_t *ref_v,
                           int32_t n_ref, const void *cache, float *out, void *ws,
                           size_t ws_bytes, void *stream);

/* Difference of two learned fields (multi-point analysis, Sec. 6.4):
 * out[v] = Phi(p_a, p_v) - Phi(p_b, p_v) at every grid vertex v, for reference
 * vertices ref_a, ref_b in [0, V).  cache holds the query latents written by
 * ndf_infer_latents for the same qparams; ws needs
 * ndf_workspace_bytes(NDF_OP_INFER_CACHED, NULL, cfg, 2, NDF_PREC_BF16) bytes.
 * One launch reads each cached latent once and decodes both fields from it;
 * the result equals the FP32 difference of the two ndf_infer_field_cached
 * fields bit for bit.  NDF_E_ARG for a null pointer or a vertex out of range. */
int ndf_infer_field_difference(const ndf_net_config *cfg, const void *qparams, int64_t ref_a,
                               int64_t ref_b, const void *cache, float *out, void *ws,
                               size_t ws_bytes, void *stream);

/* The learned field at arbitrary sample positions instead of grid vertices (the
 * positions a ray marcher visits, Sec. 5; the network's input domain of
 * Sec. 4.3): out[r][i] = Phi(p_ref[r], pos[i]) for ref_v [host] int64[n_ref]
 * vertices and pos float[n][3] (device, x y z per position) in the domain
 * [-1, 1]^3, where -1 and +1 are the first and last grid vertex of an axis
 * (vertex (i, j, k) sits at 2 i/(nx - 1) - 1, ...).  Each grid level is
 * interpolated trilinearly at the position; coordinates outside the domain are
 * clamped to its boundary, NaN coordinates to -1.  out float[n_ref][n] (device).
 * prec, qparams and ws as for ndf_infer_field.  n = 0 enqueues nothing.
 * NDF_E_ARG for null pointers, n < 0, n_ref < 1 or a reference out of range. */
int ndf_infer_points(const ndf_net_config *cfg, const void *qparams, int32_t prec,
                     const int64_t *ref_v, int32_t n_ref, const float *pos, int64_t n, float *out,
                     void *ws, size_t ws_bytes, void *stream);

/* Phi(p1, p2) for B vertex pairs (device int64[B][2]) from the FP32 parameters
 * with the training forward kernels (BF16 MFMA, FP32 accumulate); y float[B]. */
int ndf_net_forward(const ndf_net_config *cfg, const float *params, const int64_t *pairs,
                    int64_t B, float *y, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NDF_H */
