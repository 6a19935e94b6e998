// Direct KSG mutual-information dependence (Sec. 3.2, Eq. 2; nearest-neighbour
// estimator of Kraskov, Stoegbauer and Grassberger, their first algorithm).
//
// For one (reference a, query b) pair the N samples are (x_m, y_m) =
// (code[a][m], code[b][m]), integer codes from ndf_prepare.  For every sample
//   eps_m = k-th smallest max(|x_m - x_j|, |y_m - y_j|) over j != m,
//   nx_m  = #{j != m : |x_m - x_j| < eps_m},  ny_m likewise in y,
// and I = psi(k) + psi(N) - <psi(nx+1) + psi(ny+1)>, which with
// psi(n) = H_{n-1} - gamma is H_{k-1} + H_{N-1} - <H_nx + H_ny>.
//
// GPU design (one workgroup of four 64-lane waves per pair, everything in LDS;
// four waves share one pair's LDS so that a CU keeps enough waves in flight to
// hide LDS latency):
//  * the samples are kept in two orders, by x and by y; both come from the
//    per-vertex sorted member orders that ndf_prepare stores (ties by member
//    index), so no query sorts anything; without stored orders every column is
//    sorted on the fly (ties by member index in x, by x position in y), which
//    gives bit-identical results;
//  * the k nearest neighbours of a sample are found by walking outwards from its
//    own position in one of the two orders, stopping on each side once the
//    distance along that coordinate reaches the current k-th distance (under the
//    max-norm no later sample can be closer).  Each sample walks the order in
//    which its 2k nearest codes are spread widest, i.e. where the strip the walk
//    must cover holds the fewest samples; any choice gives the same exact result;
//  * the marginal counts are two lower bounds each, over the sorted x codes and
//    over the sorted y codes; a bucket table of each order (built per pair in
//    LDS) narrows every search to the few samples of one code bucket;
//  * all distances and counts are exact int32, so the counts equal a brute-force
//    evaluation bit for bit; the harmonic sum is FP64.
#include "common.hpp"

namespace ndf {

constexpr int kKsgMaxN = 4096;
constexpr int kKsgWaves = 4;
constexpr int kKsgThreads = 64 * kKsgWaves;

__device__ __forceinline__ int pow2_ceil(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Ascending bitonic sort of P (power of two) keys in LDS by the workgroup.
template <typename T>
__device__ void block_bitonic_sort(T *a, int P) {
    const int tid = threadIdx.x;
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += kKsgThreads) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                T u = a[i], w = a[j];
                if ((u > w) == up) {
                    a[i] = w;
                    a[j] = u;
                }
            }
            __syncthreads();
        }
    }
}

// Bucket tables of the marginal searches: T[b] = number of sorted codes below
// b * 2^kTabShift for b = 0 .. kTabN - 1 (codes lie in [0, 2^23], so the last
// entry is N).  A lower bound of v then only searches [T[b], T[b + 1]] with
// b = v >> kTabShift: a handful of samples instead of all N.
constexpr int kTabShift = 14;
constexpr int kTabN = ((1 << 23) >> kTabShift) + 2;  // 514 entries

__device__ __forceinline__ int tab_bucket(int v) {
    return min(max(v, 0) >> kTabShift, kTabN - 2);
}

// Table construction in three steps with a workgroup barrier between them:
// every entry N (all threads) ...
__device__ __forceinline__ void tab_fill(uint16_t *T, int N) {
    for (int i = threadIdx.x; i < kTabN; i += kKsgThreads) T[i] = (uint16_t)N;
}
// ... the first position of every non-empty bucket of the sorted a[0..N) (all
// threads) ...
__device__ __forceinline__ void tab_scatter(const int2 *a, uint16_t *T, int N) {
    for (int j = threadIdx.x; j < N; j += kKsgThreads) {
        const int b = tab_bucket(a[j].x);
        if (j == 0 || tab_bucket(a[j - 1].x) != b) T[b] = (uint16_t)j;
    }
}
// ... and a suffix minimum by one wave, so that an empty bucket takes the first
// position of the next non-empty one (lane l owns entries kPer l .. kPer l + kPer - 1).
__device__ __forceinline__ void tab_scan(uint16_t *T) {
    constexpr int kPer = (kTabN + 63) / 64;
    const int lane = threadIdx.x & 63;
    int v[kPer];
    int run = 0xffff;
#pragma unroll
    for (int i = kPer - 1; i >= 0; --i) {
        const int idx = lane * kPer + i;
        if (idx < kTabN) run = min(run, (int)T[idx]);
        v[i] = run;
    }
    int s = run;  // minimum over the chunks of this lane and all later ones
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_down(s, d);
        if (lane + d < 64) s = min(s, t);
    }
    int carry = __shfl_down(s, 1);
    if (lane == 63) carry = 0xffff;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int idx = lane * kPer + i;
        if (idx < kTabN) T[idx] = (uint16_t)min(v[i], carry);
    }
}

// Marginal counts of one sample with k-th distance eps > 0: entries of the sorted
// x codes (xo[].x) and of the sorted y codes (yo[].x) strictly inside
// (v - eps, v + eps), minus the sample itself.  Each of the four lower bounds
// starts from its bucket range [T[b], T[b + 1]]; the searches advance in lockstep
// from the widest range's step, so their LDS reads are in flight together, and a
// probe is clamped into [0, N) and never advances past its range.
__device__ __forceinline__ void marginal_counts(const int2 *xo, const int2 *yo,
                                                const uint16_t *Tx, const uint16_t *Ty, int N,
                                                int2 mxy, int eps, int &nx, int &ny) {
    const int val[4] = {mxy.x + eps, mxy.x - eps + 1, mxy.y + eps, mxy.y - eps + 1};
    int pos[4], hi[4], span = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint16_t *T = i < 2 ? Tx : Ty;
        const int b = tab_bucket(val[i]);
        pos[i] = T[b];
        hi[i] = T[b + 1];
        span = max(span, hi[i] - pos[i]);
    }
    for (int st = span > 0 ? 1 << (31 - __clz(span)) : 0; st > 0; st >>= 1) {
        int c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = (i < 2 ? xo : yo)[min(pos[i] + st, N) - 1].x;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (pos[i] + st <= hi[i] && c[i] < val[i]) pos[i] += st;
    }
    nx = pos[0] - pos[1] - 1;
    ny = pos[2] - pos[3] - 1;
}

constexpr int kPad = 4;             // sentinel samples on each side of the x order
constexpr int kFar = 1 << 29;       // sentinel x: its distance to any sample exceeds kUnset
constexpr int kUnset = 1 << 28;     // k-th distance before k samples are seen: above any
                                    // code difference (< 2^24), below any sentinel distance

// v_med3_i32: the middle of three signed integers.  With lo <= hi it is d
// clamped to [lo, hi] in one instruction (the compiler forms it only for
// constant bounds).  Operands are plain VALU results, so the asm needs no wait
// states.
__device__ __forceinline__ int med3_i32(int d, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(d), "v"(lo), "v"(hi));
    return r;
}

// |a - b| of two codes (both in [0, 2^24)) in one v_sad_u32.
__device__ __forceinline__ int absdiff_u32(int a, int b) {
    int r;
    asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <int K>
__device__ __forceinline__ void insert_k(int (&best)[K], int d) {
    // best ascending; keep the K smallest of best + {d} (ties kept with
    // multiplicity): best[t] = min(best[t], max(best[t - 1], d)) = d clamped
    // to [best[t - 1], best[t]]
#pragma unroll
    for (int t = K - 1; t > 0; --t) best[t] = med3_i32(d, best[t - 1], best[t]);
    best[0] = min(best[0], d);
}

// Neighbour search and counts for all samples of one pair.
//   xo[p] = (x, y) in x order, yo[q] = (y, x) in y order, both with kPad
//   sentinels on each side; yrank[p] = y-order position of x-order sample p;
//   perm[p] = member of x-order sample p; epsL = N ints of LDS scratch;
//   Tx, Ty = bucket tables of the x and y orders, every entry N on entry (Tx
//   already built unless build_tx), every entry N again on return.
// Returns the FP64 sum of H_nx + H_ny over all samples.
//
// Walk phase: first every sample's walk order and start position are computed
// with all lanes busy.  Then the x order is dealt to the waves in chunks of 64
// samples, round robin.  A lane walks one sample at a time; once 16 lanes of the
// wave have finished, they take the wave's next unclaimed samples (handed out in
// lane order from a wave-uniform counter), so short and long walks do not wait
// for each other.
// A walk takes 4 samples per side per step; a side stops once the farthest of
// its 4 is at least the current k-th distance away along the walked coordinate
// (always so for a sentinel, as the k-th distance starts at kUnset).  Samples
// past that point never change the k smallest, so the overscan is harmless; a
// block starts at most 3 samples past the last real one, and a stopped side
// reads the 4 sentinels at its end, so reads stay within the padding.
// Count phase: thread t takes samples t, t + 256, ... and counts the marginals
// by bucket table and binary search; the partial sums are combined in a fixed
// order, so the FP64 total is reproducible.  Returns the total in every thread.
template <int K>
__device__ double ksg_points(const int2 *xo, const int2 *yo, const uint16_t *yrank, int N,
                             const double *__restrict__ H, const uint16_t *perm,
                             int32_t *__restrict__ cnt, int *epsL, uint16_t *Tx, uint16_t *Ty,
                             bool build_tx) {
    __shared__ double s_part[kKsgWaves];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // i-th sample of this wave (increasing in i)
    auto sample = [&](int i) { return ((i >> 6) * kKsgWaves + wave) * 64 + (i & 63); };
    int p = sample(lane);
    bool active = false;
    const int2 *A = xo;
    const int2 *L = xo, *R = xo;  // next blocks: L[0..3] left (farthest first), R[0..3] right
    int2 me = make_int2(0, 0);
    int best[K];
#pragma unroll
    for (int t = 0; t < K; ++t) best[t] = kUnset;

    // Every sample's walk order and start position, with all lanes busy:
    // epsL[p] = position | (walk in y order) << 16 until the walk of p ends.
    for (int pp = tid; pp < N; pp += kKsgThreads) {
        const int q = min((int)yrank[pp], N - 1);
        // spread of the 32 nearest codes in each order: walk the sparser one (a
        // wider window than the k nearest predicts the walk's strip better: 4 %
        // fewer walk steps than with 2k on the synthetic ensembles)
        constexpr int W = 16;
        const int sx = xo[min(pp + W, N - 1)].x - xo[max(pp - W, 0)].x;
        const int sy = yo[min(q + W, N - 1)].x - yo[max(q - W, 0)].x;
        epsL[pp] = sy > sx ? (q | 0x10000) : pp;
    }
    tab_scatter(yo, Ty, N);
    if (build_tx) tab_scatter(xo, Tx, N);
    __syncthreads();
    if (wave == 0)
        tab_scan(Ty);
    else if (wave == 1 && build_tx)
        tab_scan(Tx);

    auto start = [&](int pp) {
        const int info = epsL[pp];
        A = info >= 0x10000 ? yo : xo;
        // a walk starts inside the sentinel-padded order, so it ends at a
        // sentinel at the latest, whatever the data
        const int pos = min(info & 0xffff, N - 1);
        me = A[pos];  // the sample itself in its walk order: (walked, other)
        L = A + pos - 4;
        R = A + pos + 1;
#pragma unroll
        for (int t = 0; t < K; ++t) best[t] = kUnset;
    };

    if (p < N) {
        start(p);
        active = true;
    }
    int next = 64;  // first unclaimed sample (wave-uniform)
    bool more = sample(next) < N;
    for (;;) {
        if (active) {
            // Both sides every step, no branches: a finished side reads the
            // sentinel block at its end of the order, whose distances exceed
            // every k-th distance, so it changes nothing.
            int2 c[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = L[u];
                c[4 + u] = R[u];
            }
#pragma unroll
            for (int u = 3; u >= 0; --u)
                insert_k<K>(best, max(me.x - c[u].x, absdiff_u32(me.y, c[u].y)));
#pragma unroll
            for (int u = 0; u < 4; ++u)
                insert_k<K>(best, max(c[4 + u].x - me.x, absdiff_u32(me.y, c[4 + u].y)));
            // a side goes on while its farthest sample is nearer than the k-th
            // distance (never for a sentinel, never past the padding)
            const bool al = (me.x - c[0].x) < best[K - 1];
            const bool ar = (c[7].x - me.x) < best[K - 1];
            L = al ? L - 4 : A - kPad;
            R = ar ? R + 4 : A + N;
            if (!al && !ar) {
                epsL[p] = best[K - 1];
                active = false;
            }
        }
        const uint64_t idle = __ballot(!active);
        if (!more) {
            if (idle == ~0ull) break;
            continue;
        }
        // refill once a quarter of the lanes is idle: the claim code runs with
        // only the idle lanes on, so batching claims costs fewer issue slots than
        // the short idle wait (measured: 51.3 ms refilling at every step, 50.5 ms
        // at 16 idle lanes, 52.2 ms at 32)
        if (__popcll(idle) < 16) continue;
        if (!active) {
            // rank of this lane among the idle ones
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0));
            const int np = sample(next + rank);
            if (np < N) {
                p = np;
                start(p);
                active = true;
            }
        }
        next = __builtin_amdgcn_readfirstlane(next + __popcll(idle));
        more = sample(next) < N;
    }
    __syncthreads();

    double acc = 0.0;
    for (int pp = tid; pp < N; pp += kKsgThreads) {
        const int2 mxy = xo[pp];
        const int eps = epsL[pp];
        int nx = 0, ny = 0;
        if (eps > 0) marginal_counts(xo, yo, Tx, Ty, N, mxy, eps, nx, ny);
        nx = min(max(nx, 0), N - 1);  // no-ops on sorted orders; keep H reads in bounds
        ny = min(max(ny, 0), N - 1);
        acc += H[nx] + H[ny];
        if (cnt) {
            const int m = perm[pp];
            cnt[m] = nx;
            cnt[N + m] = ny;
        }
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) s_part[wave] = acc;
    __syncthreads();
    double total = 0.0;
#pragma unroll
    for (int w = 0; w < kKsgWaves; ++w) total += s_part[w];
    tab_fill(Ty, N);  // for the next pair (the counts above were the last readers)
    if (build_tx) tab_fill(Tx, N);
    return total;
}

// Ascending bitonic sort of 256 E keys held E per thread in registers (thread t
// holds keys E t .. E t + E - 1).  Compare-exchange partners closer than E are in
// the thread's own registers, partners up to 64 E apart are in the same wave
// (lane shuffles), and only the strides of 64 E and more go through LDS (xchg,
// 256 E keys), so a sort of 1024 keys takes 3 workgroup barriers instead of 55.
template <int E>
__device__ __forceinline__ void block_sort_regs(unsigned long long (&k)[E],
                                                unsigned long long *xchg) {
    const int tid = threadIdx.x;
    constexpr int PT = kKsgThreads * E;
    for (int size = 2; size <= PT; size <<= 1) {
        for (int stride = size >> 1; stride >= E; stride >>= 1) {
            const bool cross = stride >= 64 * E;
            if (cross) {
                __syncthreads();
#pragma unroll
                for (int j = 0; j < E; ++j) xchg[E * tid + j] = k[j];
                __syncthreads();
            }
            // the lower index of a pair keeps the smaller key in an ascending
            // block; stride >= E, so that is the same for all E keys of a thread
            const bool keep_min = ((E * tid & stride) == 0) == ((E * tid & size) == 0);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int i = E * tid + j;
                const unsigned long long o =
                    cross ? xchg[i ^ stride] : __shfl_xor(k[j], stride / E, kWave);
                // equal keys are interchangeable, so one comparison decides
                k[j] = ((o < k[j]) == keep_min) ? o : k[j];
            }
        }
#pragma unroll
        for (int st = E / 2; st >= 1; st >>= 1) {
            if (st >= size) continue;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int jp = j ^ st;
                if (jp < j) continue;
                const bool up = ((E * tid + j) & size) == 0;
                const unsigned long long a = k[j], b = k[jp];
                const bool swap = (a > b) == up;
                k[j] = swap ? b : a;
                k[jp] = swap ? a : b;
            }
        }
    }
    __syncthreads();  // xchg may be reused by the caller
}

// The y order from a complete x order: (y, x position) keys sorted in
// registers, written out as yo[q] = (y, x) with each sample's y rank.  The
// exchange buffer of the sort is the yo region itself.
template <int E>
__device__ __forceinline__ void build_y_order_e(int2 *xo, int2 *yo, uint16_t *yrank, int N) {
    const int tid = threadIdx.x;
    unsigned long long k[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = E * tid + j;
        k[j] = p < N ? (((unsigned long long)(uint32_t)xo[p].y) << 32) | (unsigned)p : ~0ull;
    }
    block_sort_regs<E>(k, reinterpret_cast<unsigned long long *>(yo));
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int q = E * tid + j;
        if (q < N) {
            const int p = (int)(k[j] & 0xffffffffu);
            yo[q] = make_int2((int)(k[j] >> 32), xo[p].x);
            yrank[p] = (uint16_t)q;
        }
    }
    if (tid < kPad) {
        yo[-1 - tid] = make_int2(-kFar, 0);
        yo[N + tid] = make_int2(kFar, 0);
    }
    __syncthreads();
}

// The x order of a pair from its two code rows: (x code, member) keys sorted in
// registers, written out as xo[p] = (x, y) and perm[p] = member (exchange buffer:
// the yo region).
template <int E>
__device__ __forceinline__ void build_x_order_e(const int32_t *__restrict__ ca,
                                                const int32_t *__restrict__ cb, int N, int2 *xo,
                                                uint16_t *perm, int2 *yo) {
    const int tid = threadIdx.x;
    unsigned long long k[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int m = E * tid + j;
        k[j] = m < N ? (((unsigned long long)(uint32_t)ca[m]) << 16) | (unsigned)m : ~0ull;
    }
    block_sort_regs<E>(k, reinterpret_cast<unsigned long long *>(yo));
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = E * tid + j;
        if (p < N) {
            const int m = (int)(k[j] & 0xffff);
            perm[p] = (uint16_t)m;
            xo[p] = make_int2((int)(k[j] >> 16), cb[m]);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void build_x_order(const int32_t *__restrict__ ca,
                                              const int32_t *__restrict__ cb, int N, int P,
                                              int2 *xo, uint16_t *perm, int2 *yo) {
    if (P <= kKsgThreads)
        build_x_order_e<1>(ca, cb, N, xo, perm, yo);
    else if (P <= 2 * kKsgThreads)
        build_x_order_e<2>(ca, cb, N, xo, perm, yo);
    else if (P <= 4 * kKsgThreads)
        build_x_order_e<4>(ca, cb, N, xo, perm, yo);
    else {  // N > 1024: sort in LDS (8 keys per thread in registers would cost occupancy)
        const int tid = threadIdx.x;
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(yo);
        for (int m = tid; m < P; m += kKsgThreads)
            keys[m] = m < N ? (((unsigned long long)(uint32_t)ca[m]) << 16) | (unsigned)m : ~0ull;
        __syncthreads();
        block_bitonic_sort(keys, P);
        for (int p = tid; p < N; p += kKsgThreads) {
            const int m = (int)(keys[p] & 0xffff);
            perm[p] = (uint16_t)m;
            xo[p] = make_int2((int)(keys[p] >> 16), cb[m]);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void build_y_order(int2 *xo, int2 *yo, uint16_t *yrank, int N, int P) {
    if (P <= kKsgThreads)
        build_y_order_e<1>(xo, yo, yrank, N);
    else if (P <= 2 * kKsgThreads)
        build_y_order_e<2>(xo, yo, yrank, N);
    else if (P <= 4 * kKsgThreads)
        build_y_order_e<4>(xo, yo, yrank, N);
    else {  // N > 1024: sort in LDS
        const int tid = threadIdx.x;
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(yo);
        for (int p = tid; p < P; p += kKsgThreads)
            keys[p] = p < N ? (((unsigned long long)(uint32_t)xo[p].y) << 32) | (unsigned)p : ~0ull;
        __syncthreads();
        block_bitonic_sort(keys, P);
        for (int q = tid; q < N; q += kKsgThreads) {
            const unsigned long long key = keys[q];
            const int p = (int)(key & 0xffffffffu);
            yo[q] = make_int2((int)(key >> 32), xo[p].x);
            yrank[p] = (uint16_t)q;
        }
        __syncthreads();
        if (tid < kPad) {
            yo[-1 - tid] = make_int2(-kFar, 0);
            yo[N + tid] = make_int2(kFar, 0);
        }
        __syncthreads();
    }
}

// Sentinels of the x order (written once per launch by each workgroup).
__device__ __forceinline__ void ksg_sentinels(int2 *xy, int N) {
    const int tid = threadIdx.x;
    if (tid < kPad) {
        xy[-1 - tid] = make_int2(-kFar, 0);
        xy[N + tid] = make_int2(kFar, 0);
    }
}

// ----------------------------------------------------------- field mode ----
// Prologue: for each reference, its codes in ascending (code, member) order and
// the member permutation; plus the harmonic table H[0..N] (sequential FP64 sum).
__global__ void ksg_sort_ref_kernel(const int32_t *__restrict__ code,
                                    const uint16_t *__restrict__ order, int N,
                                    const int64_t *__restrict__ refs, int32_t *__restrict__ xs,
                                    uint16_t *__restrict__ perm, uint16_t *__restrict__ invp,
                                    double *__restrict__ H) {
    extern __shared__ unsigned long long s_keys[];
    const int r = blockIdx.x;
    const int P = pow2_ceil(N);
    const int32_t *c = code + refs[r] * N;
    if (order) {  // the column's stored order
        const uint16_t *o = order + refs[r] * N;
        for (int p = threadIdx.x; p < N; p += kKsgThreads) {
            const int m = min((int)o[p], N - 1);  // in bounds even if never prepared
            xs[(int64_t)r * N + p] = c[m];
            perm[(int64_t)r * N + p] = (uint16_t)m;
            invp[(int64_t)r * N + m] = (uint16_t)p;
        }
    } else {
        for (int m = threadIdx.x; m < P; m += kKsgThreads)
            s_keys[m] = m < N ? (((unsigned long long)(uint32_t)c[m]) << 16) | (unsigned)m : ~0ull;
        __syncthreads();
        block_bitonic_sort(s_keys, P);
        for (int p = threadIdx.x; p < N; p += kKsgThreads) {
            const int m = (int)(s_keys[p] & 0xffff);
            xs[(int64_t)r * N + p] = (int32_t)(s_keys[p] >> 16);
            perm[(int64_t)r * N + p] = (uint16_t)m;
            invp[(int64_t)r * N + m] = (uint16_t)p;
        }
    }
    if (r == 0 && threadIdx.x == 0) {
        double h = 0.0;
        H[0] = 0.0;
        for (int i = 1; i <= N; ++i) {
            h += 1.0 / (double)i;
            H[i] = h;
        }
    }
}

// Every column's members in ascending (code, member) order: the sorted orders of
// the neighbour search, built once per ensemble.  Workgroups stride over the
// columns (one per wave for N <= 1024, else one per workgroup).
template <int E>
__device__ __forceinline__ void sort_column_e(const int32_t *__restrict__ c, int N,
                                              uint16_t *__restrict__ o,
                                              unsigned long long *xchg) {
    const int tid = threadIdx.x;
    unsigned long long k[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int m = E * tid + j;
        k[j] = m < N ? (((unsigned long long)(uint32_t)c[m]) << 16) | (unsigned)m : ~0ull;
    }
    block_sort_regs<E>(k, xchg);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = E * tid + j;
        if (p < N) o[p] = (uint16_t)(k[j] & 0xffff);
    }
}

// One wave sorts 64 E keys held E per lane (lane l holds keys E l .. E l + E - 1):
// partners closer than E are in the lane's registers, all others are lane
// shuffles; no LDS and no barrier.
template <int E>
__device__ __forceinline__ void wave_sort_regs(unsigned long long (&k)[E]) {
    const int lane = threadIdx.x & 63;
    constexpr int PT = 64 * E;
    for (int size = 2; size <= PT; size <<= 1) {
        for (int stride = size >> 1; stride >= E; stride >>= 1) {
            const bool keep_min = ((E * lane & stride) == 0) == ((E * lane & size) == 0);
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const unsigned long long o = __shfl_xor(k[j], stride / E, kWave);
                k[j] = ((o < k[j]) == keep_min) ? o : k[j];
            }
        }
#pragma unroll
        for (int st = E / 2; st >= 1; st >>= 1) {
            if (st >= size) continue;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int jp = j ^ st;
                if (jp < j) continue;
                const bool up = ((E * lane + j) & size) == 0;
                const unsigned long long a = k[j], b = k[jp];
                const bool swap = (a > b) == up;
                k[j] = swap ? b : a;
                k[jp] = swap ? a : b;
            }
        }
    }
}

// Ascending bitonic sort of 64 E 32-bit keys held E per lane, in the form whose
// merge of two sorted halves starts by comparing element i with its mirror
// i ^ (size - 1): every comparator then puts the minimum at the lower index, so a
// pair in one lane is one v_min and one v_max, and a pair across lanes one lane
// shuffle plus a min or max.
template <int E>
__device__ __forceinline__ void wave_sort_regs32(uint32_t (&k)[E]) {
    const int lane = threadIdx.x & 63;
    constexpr int LE = E == 1 ? 0 : E == 2 ? 1 : E == 4 ? 2 : E == 8 ? 3 : 4;
    constexpr int LPT = 6 + LE;  // log2 of the key count
#pragma unroll
    for (int ls = 1; ls <= LPT; ++ls) {
        const int size = 1 << ls;
        if (size <= E) {
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const int jp = j ^ (size - 1);
                if (jp > j) {
                    const uint32_t a = k[j], b = k[jp];
                    k[j] = min(a, b);
                    k[jp] = max(a, b);
                }
            }
        } else {
            // partner of (lane, j) is (lane ^ (size / E - 1), E - 1 - j)
            const bool lower = ((E * lane) & (size >> 1)) == 0;
            uint32_t t[E];
#pragma unroll
            for (int j = 0; j < E; ++j) t[j] = __shfl_xor(k[E - 1 - j], size / E - 1, kWave);
#pragma unroll
            for (int j = 0; j < E; ++j) k[j] = lower ? min(k[j], t[j]) : max(k[j], t[j]);
        }
#pragma unroll
        for (int ls2 = ls - 2; ls2 >= 0; --ls2) {
            const int stride = 1 << ls2;
            if (stride >= E) {
                const bool lower = ((E * lane) & stride) == 0;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const uint32_t o = __shfl_xor(k[j], stride / E, kWave);
                    k[j] = lower ? min(k[j], o) : max(k[j], o);
                }
            } else {
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int jp = j ^ stride;
                    if (jp > j) {
                        const uint32_t a = k[j], b = k[jp];
                        k[j] = min(a, b);
                        k[jp] = max(a, b);
                    }
                }
            }
        }
    }
}

// Sorted member order of one column with 64 < N <= 1024 (E >= 2 per lane).  The
// sort runs on 32-bit keys (code >> 2, member): codes lie in [0, 2^23], so
// code >> 2 takes 22 bits and the member 10.  Samples whose codes agree above
// the two lowest bits then sit in member order; where such neighbours exist,
// odd-even transposition passes on the full (code, member) keys finish the
// order, and a column that is still unsorted after four rounds (many near-equal
// codes) is sorted again on full 64-bit keys.
template <int E>
__device__ __forceinline__ void wave_sort_column32(const int32_t *__restrict__ c, int N,
                                                   uint16_t *__restrict__ o) {
    static_assert(E >= 2, "pairs of one lane");
    const int lane = threadIdx.x & 63;
    uint32_t k[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int m = E * lane + j;
        k[j] = m < N ? (((uint32_t)c[m] >> 2) << 10) | (uint32_t)m : 0xffffffffu;
    }
    wave_sort_regs32<E>(k);
    // neighbours with equal code >> 2 (padding keys never tie with a sample)
    bool tie = false;
#pragma unroll
    for (int j = 0; j + 1 < E; ++j) tie |= (k[j] >> 10) == (k[j + 1] >> 10) && k[j + 1] != 0xffffffffu;
    const uint32_t nk = __shfl_down(k[0], 1, kWave);
    if (lane < 63) tie |= (k[E - 1] >> 10) == (nk >> 10) && nk != 0xffffffffu;
    if (!__any(tie)) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int p = E * lane + j;
            if (p < N) o[p] = (uint16_t)(k[j] & 0x3ff);
        }
        return;
    }
    unsigned long long f[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int m = (int)(k[j] & 0x3ff);
        f[j] = k[j] == 0xffffffffu ? ~0ull
                                   : (((unsigned long long)(uint32_t)c[m]) << 16) | (unsigned)m;
    }
    auto in_order = [&]() {
        bool bad = false;
#pragma unroll
        for (int j = 0; j + 1 < E; ++j) bad |= f[j] > f[j + 1];
        const unsigned long long nf = __shfl_down(f[0], 1, kWave);
        if (lane < 63) bad |= f[E - 1] > nf;
        return !__any(bad);
    };
    bool done = false;
    for (int round = 0; round < 4 && !(done = in_order()); ++round) {
#pragma unroll
        for (int j = 0; j + 1 < E; j += 2) {  // pairs (2i, 2i + 1)
            const unsigned long long a = f[j], b = f[j + 1];
            f[j] = a < b ? a : b;
            f[j + 1] = a < b ? b : a;
        }
        const unsigned long long nf = __shfl_down(f[0], 1, kWave);
        const unsigned long long pf = __shfl_up(f[E - 1], 1, kWave);
#pragma unroll
        for (int j = 1; j + 1 < E; j += 2) {  // pairs (2i + 1, 2i + 2) inside a lane
            const unsigned long long a = f[j], b = f[j + 1];
            f[j] = a < b ? a : b;
            f[j + 1] = a < b ? b : a;
        }
        // the pair across a lane boundary: the lower position keeps the minimum
        if (lane < 63) f[E - 1] = f[E - 1] < nf ? f[E - 1] : nf;
        if (lane > 0) f[0] = f[0] > pf ? f[0] : pf;
    }
    if (!done && !in_order()) wave_sort_regs<E>(f);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = E * lane + j;
        if (p < N) o[p] = (uint16_t)(f[j] & 0xffff);
    }
}

template <int E>
__device__ __forceinline__ void wave_sort_column(const int32_t *__restrict__ c, int N,
                                                 uint16_t *__restrict__ o) {
    const int lane = threadIdx.x & 63;
    unsigned long long k[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int m = E * lane + j;
        k[j] = m < N ? (((unsigned long long)(uint32_t)c[m]) << 16) | (unsigned)m : ~0ull;
    }
    wave_sort_regs<E>(k);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = E * lane + j;
        if (p < N) o[p] = (uint16_t)(k[j] & 0xffff);
    }
}

__global__ __launch_bounds__(kKsgThreads) __attribute__((amdgpu_waves_per_eu(4))) void ksg_order_kernel(const int32_t *__restrict__ code,
                                                                int N, int64_t ncol,
                                                                uint16_t *__restrict__ order) {
    extern __shared__ unsigned long long s_x[];
    const int P2 = pow2_ceil(N);
    if (P2 <= 1024) {  // one column per wave
        const int64_t waves = (int64_t)gridDim.x * kKsgWaves;
        for (int64_t v = (int64_t)blockIdx.x * kKsgWaves + (threadIdx.x >> 6); v < ncol;
             v += waves) {
            const int32_t *c = code + v * N;
            uint16_t *o = order + v * N;
            if (P2 <= 64)
                wave_sort_column<1>(c, N, o);
            else if (P2 <= 128)
                wave_sort_column32<2>(c, N, o);
            else if (P2 <= 256)
                wave_sort_column32<4>(c, N, o);
            else if (P2 <= 512)
                wave_sort_column32<8>(c, N, o);
            else
                wave_sort_column32<16>(c, N, o);
        }
        return;
    }
    const int P = max(P2, kKsgThreads);
    for (int64_t v = blockIdx.x; v < ncol; v += gridDim.x) {
        const int32_t *c = code + v * N;
        uint16_t *o = order + v * N;
        if (P <= kKsgThreads)
            sort_column_e<1>(c, N, o, s_x);
        else if (P <= 2 * kKsgThreads)
            sort_column_e<2>(c, N, o, s_x);
        else if (P <= 4 * kKsgThreads)
            sort_column_e<4>(c, N, o, s_x);
        else {
            for (int m = threadIdx.x; m < P; m += kKsgThreads)
                s_x[m] = m < N ? (((unsigned long long)(uint32_t)c[m]) << 16) | (unsigned)m : ~0ull;
            __syncthreads();
            block_bitonic_sort(s_x, P);
            for (int p = threadIdx.x; p < N; p += kKsgThreads) o[p] = (uint16_t)(s_x[p] & 0xffff);
            __syncthreads();
        }
    }
}

// LDS plan of both kernels: xo (N + 2 kPad) int2 | yo (P + 2 kPad) int2, also the
// sort keys and exchange buffer | perm N uint16 | yrank N uint16 | eps N int32 |
// Tx, Ty kTabN uint16 each, with P = max(pow2_ceil(N), 256) (the register sort
// always moves 256 E keys).
__host__ __device__ inline size_t ksg_lds_bytes(int N, int P) {
    return (size_t)(N + 2 * kPad) * 8 + (size_t)(P + 2 * kPad) * 8 + (size_t)N * 4 +
           (size_t)N * 4 + (size_t)kTabN * 4;
}

template <int K>
__global__ __launch_bounds__(kKsgThreads) __attribute__((amdgpu_waves_per_eu(6))) void ksg_field_kernel(
    const int32_t *__restrict__ code_q, const int32_t *__restrict__ flags_r,
    const int32_t *__restrict__ flags_q, int N, int64_t V, const int64_t *__restrict__ refs,
    int n_ref, const int32_t *__restrict__ xs_all, const uint16_t *__restrict__ perm_all,
    const double *__restrict__ H, float *__restrict__ out, int32_t *__restrict__ counts,
    const int32_t *__restrict__ code_r, const uint16_t *__restrict__ order_q,
    const uint16_t *__restrict__ invp_all) {
    extern __shared__ int4 s_raw[];
    const int P = max(pow2_ceil(N), kKsgThreads);  // y-order region
    int2 *xo = reinterpret_cast<int2 *>(s_raw) + kPad;
    int2 *yo = xo + N + 2 * kPad;
    uint16_t *perm = reinterpret_cast<uint16_t *>(yo + P + kPad);
    uint16_t *yrank = perm + N;
    int *epsL = reinterpret_cast<int *>(yrank + N);  // 4-byte aligned: N uint16 x 2
    uint16_t *Tx = reinterpret_cast<uint16_t *>(epsL + N);
    uint16_t *Ty = Tx + kTabN;
    int *tmp = reinterpret_cast<int *>(yo);  // the query row in member order
    const int tid = threadIdx.x;
    const double base = H[K - 1] + H[N - 1];
    ksg_sentinels(xo, N);
    tab_fill(Ty, N);

    for (int r = 0; r < n_ref; ++r) {
        const int32_t fr = flags_r[refs[r]];
        __syncthreads();
        for (int p = tid; p < N; p += kKsgThreads) {
            xo[p].x = xs_all[(int64_t)r * N + p];
            perm[p] = perm_all[(int64_t)r * N + p];
        }
        tab_fill(Tx, N);
        __syncthreads();
        // the reference's bucket table, shared by all its queries
        tab_scatter(xo, Tx, N);
        __syncthreads();
        if (tid < 64) tab_scan(Tx);
        __syncthreads();
        for (int64_t q = blockIdx.x; q < V; q += gridDim.x) {
            const int32_t *cq = code_q + q * N;
            const int32_t fq = flags_q[q];
            int32_t *cnt = counts ? counts + ((int64_t)r * V + q) * 2 * N : nullptr;
            if ((fr | fq) & (NDF_FLAG_CONSTANT | NDF_FLAG_NONFINITE)) {
                if (tid == 0)
                    out[(int64_t)r * V + q] = ((fr | fq) & NDF_FLAG_NONFINITE) ? __builtin_nanf("")
                                                                                : 0.0f;
                if (cnt)
                    for (int i = tid; i < 2 * N; i += kKsgThreads) cnt[i] = 0;
                continue;
            }
            if (order_q) {
                // both orders from stored ones: the query codes in x order, and the
                // query's own sorted order for (y, x) and the y ranks
                const uint16_t *oq = order_q + q * N;
                const int32_t *cr = code_r + refs[r] * N;
                const uint16_t *invp = invp_all + (int64_t)r * N;
                for (int p = tid; p < N; p += kKsgThreads) xo[p].y = cq[perm[p]];
                for (int j = tid; j < N; j += kKsgThreads) {
                    const int m = min((int)oq[j], N - 1);  // in bounds even if never prepared
                    yo[j] = make_int2(cq[m], cr[m]);
                    yrank[min((int)invp[m], N - 1)] = (uint16_t)j;
                }
                if (tid < kPad) {
                    yo[-1 - tid] = make_int2(-kFar, 0);
                    yo[N + tid] = make_int2(kFar, 0);
                }
                __syncthreads();
            } else {
                // the query's codes: one coalesced row read, permuted into x order in LDS
                for (int m = tid; m < N; m += kKsgThreads) tmp[m] = cq[m];
                __syncthreads();
                for (int p = tid; p < N; p += kKsgThreads) xo[p].y = tmp[perm[p]];
                __syncthreads();
                build_y_order(xo, yo, yrank, N, P);
            }
            const double acc =
                ksg_points<K>(xo, yo, yrank, N, H, perm, cnt, epsL, Tx, Ty, false);
            if (tid == 0) out[(int64_t)r * V + q] = (float)(base - acc / (double)N);
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------- pairs mode ----
template <int K>
__global__ __launch_bounds__(kKsgThreads) __attribute__((amdgpu_waves_per_eu(6))) void ksg_pairs_kernel(
    const int32_t *__restrict__ code_a, const int32_t *__restrict__ code_b,
    const int32_t *__restrict__ flags_a, const int32_t *__restrict__ flags_b, int N, int64_t V,
    const int64_t *__restrict__ pairs, int64_t B, const double *__restrict__ H,
    float *__restrict__ out, int32_t *__restrict__ counts, const uint16_t *__restrict__ order_a,
    const uint16_t *__restrict__ order_b) {
    extern __shared__ int4 s_raw[];
    const int P = max(pow2_ceil(N), kKsgThreads);  // y-order region
    int2 *xo = reinterpret_cast<int2 *>(s_raw) + kPad;
    int2 *yo = xo + N + 2 * kPad;
    uint16_t *perm = reinterpret_cast<uint16_t *>(yo + P + kPad);
    uint16_t *yrank = perm + N;
    int *epsL = reinterpret_cast<int *>(yrank + N);
    uint16_t *Tx = reinterpret_cast<uint16_t *>(epsL + N);
    uint16_t *Ty = Tx + kTabN;
    const int tid = threadIdx.x;
    const double base = H[K - 1] + H[N - 1];
    ksg_sentinels(xo, N);
    tab_fill(Tx, N);
    tab_fill(Ty, N);

    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        const int64_t va = pairs[2 * b], vb = pairs[2 * b + 1];
        int32_t *cnt = counts ? counts + b * 2 * N : nullptr;
        if (va < 0 || va >= V || vb < 0 || vb >= V) {  // out-of-range pair: NaN, no reads
            if (tid == 0) out[b] = __builtin_nanf("");
            if (cnt)
                for (int i = tid; i < 2 * N; i += kKsgThreads) cnt[i] = -1;
            continue;
        }
        const int32_t f = flags_a[va] | flags_b[vb];
        if (f & (NDF_FLAG_CONSTANT | NDF_FLAG_NONFINITE)) {
            if (tid == 0) out[b] = (f & NDF_FLAG_NONFINITE) ? __builtin_nanf("") : 0.0f;
            if (cnt)
                for (int i = tid; i < 2 * N; i += kKsgThreads) cnt[i] = 0;
            continue;
        }
        const int32_t *ca = code_a + va * N, *cb = code_b + vb * N;
        if (order_a) {
            // x order = a's stored order, y order = b's; epsL holds the inverse
            // x permutation until the walk
            const uint16_t *oa = order_a + va * N, *ob = order_b + vb * N;
            for (int p = tid; p < N; p += kKsgThreads) {
                const int m = min((int)oa[p], N - 1);  // in bounds even if never prepared
                perm[p] = (uint16_t)m;
                xo[p] = make_int2(ca[m], cb[m]);
                epsL[m] = p;
            }
            __syncthreads();
            for (int j = tid; j < N; j += kKsgThreads) {
                const int m = min((int)ob[j], N - 1);
                yo[j] = make_int2(cb[m], ca[m]);
                yrank[min(epsL[m], N - 1)] = (uint16_t)j;
            }
            if (tid < kPad) {
                yo[-1 - tid] = make_int2(-kFar, 0);
                yo[N + tid] = make_int2(kFar, 0);
            }
            __syncthreads();
        } else {
            build_x_order(ca, cb, N, P, xo, perm, yo);
            build_y_order(xo, yo, yrank, N, P);
        }
        const double acc = ksg_points<K>(xo, yo, yrank, N, H, perm, cnt, epsL, Tx, Ty, true);
        if (tid == 0) out[b] = (float)(base - acc / (double)N);
        __syncthreads();
    }
}

__global__ void harmonic_kernel(int N, double *H) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double h = 0.0;
        H[0] = 0.0;
        for (int i = 1; i <= N; ++i) {
            h += 1.0 / (double)i;
            H[i] = h;
        }
    }
}

// ------------------------------------------------------------ launchers ----
static int p2(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Workspace: H[0..N] | refs | x codes in x order [n_ref][N] | x-order members
// [n_ref][N] | inverse x permutation [n_ref][N].
size_t ksg_field_ws_bytes(int N, int n_ref) {
    return align_up((size_t)(N + 1) * sizeof(double), 256) +
           align_up((size_t)n_ref * sizeof(int64_t), 256) +
           align_up((size_t)n_ref * N * sizeof(int32_t), 256) +
           2 * align_up((size_t)n_ref * N * sizeof(uint16_t), 256);
}

// Grid of a striding kernel: `waves` times as many workgroups as the CUs hold at
// once given the LDS of one item (160 KB per CU), never more than there are
// items.  Items differ in cost (walk lengths) and CUs in speed, so a grid of
// only resident workgroups ends with a tail of the slowest ones; a larger grid
// lets the hardware hand the waiting workgroups to whichever CU frees up first
// (measured on the KSG field: 59.9 ms with 1 wave of workgroups, 51.3 with 16,
// 51.0 with 64).
static int ksg_grid(int64_t items, size_t lds, int waves) {
    int64_t per_cu = (int64_t)(163840 / (lds > 0 ? lds : 1));
    per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    const int64_t g = 256 * per_cu * waves;
    return (int)(items < g ? items : g);
}
constexpr int kPairWaves = 64;  // workgroup waves of the field and pairs kernels
constexpr int kOrderWaves = 16;  // of the sorted-order kernel

struct FieldArgs {
    const int32_t *cq, *fr, *fq;
    int N;
    int64_t V;
    const int64_t *refs;
    int n_ref;
    const int32_t *xs;
    const uint16_t *perm;
    const double *H;
    float *out;
    int32_t *counts;
    const int32_t *cr;
    const uint16_t *order_q, *invp;
};

template <int K>
static void launch_field_k(dim3 g, size_t lds, hipStream_t st, const FieldArgs &a) {
    hipLaunchKernelGGL(ksg_field_kernel<K>, g, dim3(kKsgThreads), lds, st, a.cq, a.fr, a.fq, a.N,
                       a.V, a.refs, a.n_ref, a.xs, a.perm, a.H, a.out, a.counts, a.cr, a.order_q,
                       a.invp);
}

// Sorted member orders of every column of every variable (ndf_prepare).
int launch_ksg_orders(const ndf_ensemble *e, hipStream_t st) {
    const int N = e->n_members;
    const int64_t ncol = (int64_t)e->n_vars * e->nx * e->ny * e->nz;
    const int P = p2(N) < kKsgThreads ? kKsgThreads : p2(N);
    const size_t lds = (size_t)P * sizeof(unsigned long long);
    hipLaunchKernelGGL(ksg_order_kernel, dim3((unsigned)ksg_grid(ncol, lds, kOrderWaves)),
                       dim3(kKsgThreads), lds, st, e->code, N, ncol, e->order);
    return status_of_launch();
}

int launch_ksg_field(const ndf_ensemble *e, int var_ref, int var_qry, const int64_t *ref_v,
                     int n_ref, int k, float *out, int32_t *counts, void *ws, hipStream_t st) {
    const int N = e->n_members;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    char *w = (char *)ws;
    double *H = (double *)w;
    w += align_up((size_t)(N + 1) * sizeof(double), 256);
    int64_t *refs = (int64_t *)w;
    w += align_up((size_t)n_ref * sizeof(int64_t), 256);
    int32_t *xs = (int32_t *)w;
    w += align_up((size_t)n_ref * N * sizeof(int32_t), 256);
    uint16_t *perm = (uint16_t *)w;
    w += align_up((size_t)n_ref * N * sizeof(uint16_t), 256);
    uint16_t *invp = (uint16_t *)w;
    if (put_refs(ref_v, n_ref, refs, st) != NDF_OK) return NDF_E_HIP;
    const int P = p2(N);
    const int32_t *cr = e->code + (int64_t)var_ref * V * N;
    const int32_t *cq = e->code + (int64_t)var_qry * V * N;
    const uint16_t *ordr = e->order ? e->order + (int64_t)var_ref * V * N : nullptr;
    const uint16_t *ordq = e->order ? e->order + (int64_t)var_qry * V * N : nullptr;
    hipLaunchKernelGGL(ksg_sort_ref_kernel, dim3(n_ref), dim3(kKsgThreads), (size_t)P * 8, st, cr,
                       ordr, N, refs, xs, perm, invp, H);
    const size_t lds = ksg_lds_bytes(N, P < kKsgThreads ? kKsgThreads : P);
    const dim3 g((unsigned)ksg_grid(V, lds, kPairWaves));
    const FieldArgs a{cq, e->flags + (int64_t)var_ref * V, e->flags + (int64_t)var_qry * V,
                      N, V, refs, n_ref, xs, perm, H, out, counts, cr, ordq, invp};
    switch (k) {
#define NDF_KSG_CASE(KK) \
    case KK: launch_field_k<KK>(g, lds, st, a); break;
        NDF_KSG_CASE(1) NDF_KSG_CASE(2) NDF_KSG_CASE(3) NDF_KSG_CASE(4)
        NDF_KSG_CASE(5) NDF_KSG_CASE(6) NDF_KSG_CASE(7) NDF_KSG_CASE(8)
#undef NDF_KSG_CASE
        default: return NDF_E_UNSUPPORTED;
    }
    return status_of_launch();
}

size_t ksg_pairs_ws_bytes(int N) { return align_up((size_t)(N + 1) * sizeof(double), 256); }

int launch_ksg_pairs(const ndf_ensemble *e, int var_a, int var_b, const int64_t *pairs, int64_t B,
                     int k, float *out, int32_t *counts, double *H, hipStream_t st) {
    const int N = e->n_members;
    const int64_t V = (int64_t)e->nx * e->ny * e->nz;
    const int P = p2(N);
    hipLaunchKernelGGL(harmonic_kernel, dim3(1), dim3(64), 0, st, N, H);
    const size_t lds = ksg_lds_bytes(N, P < kKsgThreads ? kKsgThreads : P);
    const dim3 g((unsigned)ksg_grid(B, lds, kPairWaves));
    const int32_t *ca = e->code + (int64_t)var_a * V * N;
    const int32_t *cb = e->code + (int64_t)var_b * V * N;
    const int32_t *fa = e->flags + (int64_t)var_a * V;
    const int32_t *fb = e->flags + (int64_t)var_b * V;
    const uint16_t *oa = e->order ? e->order + (int64_t)var_a * V * N : nullptr;
    const uint16_t *ob = e->order ? e->order + (int64_t)var_b * V * N : nullptr;
    switch (k) {
#define NDF_KSG_CASE(KK)                                                                       \
    case KK:                                                                                   \
        hipLaunchKernelGGL(ksg_pairs_kernel<KK>, g, dim3(kKsgThreads), lds, st, ca, cb, fa, fb, N, V, \
                           pairs, B, H, out, counts, oa, ob);                                     \
        break;
        NDF_KSG_CASE(1) NDF_KSG_CASE(2) NDF_KSG_CASE(3) NDF_KSG_CASE(4)
        NDF_KSG_CASE(5) NDF_KSG_CASE(6) NDF_KSG_CASE(7) NDF_KSG_CASE(8)
#undef NDF_KSG_CASE
        default: return NDF_E_UNSUPPORTED;
    }
    return status_of_launch();
}

}  // namespace ndf
