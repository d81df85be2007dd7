// nbody_kernels.hip -- gfx950 (CDNA4) kernels of the Hermite 6th-order block-step
// method: predictor, pairwise evaluation (FP64 and split precision), j-split
// reduction, corrector, step levels, active-set selection and energy.
//
// The paper (Goz et al., section "Code implementation") names the Hermite 6th-order
// integrator and requires double precision for inter-particle distances and
// accelerations, with an extended-precision float-float type as the alternative;
// section "Performance results" identifies the O(N^2) evaluation as the dominant
// kernel. The formulas are the standard 6th-order Hermite scheme (Nitadori &
// Makino 2008) with power-of-two block steps; each kernel states the ones it uses.
//
// Layout: body state is structure-of-arrays FP64 ([3][n] per vector); the
// predicted j-stream is an array of 80-byte records (see nb_internal.h) so a tile
// of bodies is one contiguous block, copied to LDS with 16-byte loads and read
// back as wave-uniform (broadcast) 16-byte LDS reads.
#include "nb_internal.h"
#include "nb_device.h"

#include <math.h>

namespace nb {
namespace {

__device__ __forceinline__ void raise_err(Status *stt, int word) { stt->err[word] = 1; }

// ---------------------------------------------------------------- utilities ----
template <typename T>
__global__ void k_fill(T *__restrict__ p, T v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride)
        p[i] = v;
}

__global__ void k_iota(int32_t *__restrict__ p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = i;
}

template <typename T>
hipError_t fill(T *p, T v, size_t count, hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- predictor ----
// Every body to the block time (predict_body), writing the j-records.
__global__ __launch_bounds__(256) void k_predict(Arrays A, int n, int64_t tick, double tick_size,
                                                 int split)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t ti = A.tick[i];
    if (ti > tick)
        raise_err(A.status, kErrLevel);
    const double h = (double)(tick - ti) * tick_size;
    predict_body(A.x, A.v, A.a, A.j, A.s, A.c, A.m, (size_t)n, (size_t)i, h, A.jrec,
                 split ? A.jrec32 : nullptr);
}

__global__ __launch_bounds__(256) void k_get_predicted(const double *__restrict__ jrec, int n,
                                                       double *xp, double *vp, double *ap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double *r = jrec + (size_t)i * kRecD;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (xp) xp[(size_t)k * n + i] = r[k];
        if (vp) vp[(size_t)k * n + i] = r[3 + k];
        if (ap) ap[(size_t)k * n + i] = r[6 + k];
    }
}

// j-records {x, v, a, m} of n bodies from predicted [3][n] arrays (the layout
// k_predict writes), for an evaluation of a state predicted elsewhere.
__global__ __launch_bounds__(256) void k_pack_records(const double *__restrict__ m,
                                                      const double *__restrict__ xp,
                                                      const double *__restrict__ vp,
                                                      const double *__restrict__ ap, int n,
                                                      double *__restrict__ jrec)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const size_t s = (size_t)n;
    double2 *r = reinterpret_cast<double2 *>(jrec + (size_t)i * kRecD);
    r[0] = make_double2(xp[i], xp[s + i]);
    r[1] = make_double2(xp[2 * s + i], vp[i]);
    r[2] = make_double2(vp[s + i], vp[2 * s + i]);
    r[3] = make_double2(ap[i], ap[s + i]);
    r[4] = make_double2(ap[2 * s + i], m[i]);
}

// Every value of out[count] becomes NaN if the index check of an evaluation raised
// its error word (for callers that cannot wait for the status block).
__global__ __launch_bounds__(256) void k_poison_on_index_error(const Status *__restrict__ stt,
                                                               double *__restrict__ out,
                                                               int64_t count)
{
    if (stt->err[kErrIndex] == 0)
        return;
    const double nan = __builtin_nan("");
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = nan;
}

// Start-up: the predicted accelerations become the first evaluation's a.
__global__ __launch_bounds__(256) void k_copy_acc_to_jrec(Arrays A, int n, int split)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double *r = A.jrec + (size_t)i * kRecD;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        r[6 + k] = A.evalbuf[(size_t)k * n + i];
    if (split) {
        float *f = A.jrec32 + (size_t)i * kRecF;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            f[12 + k] = (float)A.evalbuf[(size_t)k * n + i];
    }
}

// Start-up: keep the second evaluation's a, j, s (all bodies, idx = 0..n-1).
__global__ __launch_bounds__(256) void k_start_store(Arrays A, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = (size_t)k * n + i;
        A.a[e] = A.evalbuf[(size_t)(0 + k) * n + i];
        A.j[e] = A.evalbuf[(size_t)(3 + k) * n + i];
        A.s[e] = A.evalbuf[(size_t)(6 + k) * n + i];
        A.c[e] = 0.0;
        finite = finite && isfinite(A.a[e]) && isfinite(A.j[e]) && isfinite(A.s[e]);
    }
    A.phi[i] = A.evalbuf[(size_t)9 * n + i];
    A.a4n[i] = 0.0;
    A.a5n[i] = 0.0;
    // (e.g. two bodies at one place without softening)
    if (!finite || !isfinite(A.phi[i]))
        raise_err(A.status, kErrNumeric);
}

// --------------------------------------------------------- pairwise (FP64) ----
// Work decomposition: a workgroup of W waves holds W*64*IPL active bodies in
// registers (IPL per lane) and sweeps one j-range of `jchunk` bodies (one of S
// splits) tile by tile through LDS (tiles_f64). Each workgroup writes its ten
// partial sums per body to part[s][10][n_act]; k_reduce_splits adds the S splits
// in a fixed order.
template <int IPL, int NW, int TILE>
__global__ __launch_bounds__(64 * NW) void k_eval_f64(Arrays A, int n, const int32_t *__restrict__ idx,
                                                      int n_act, double eps2, int jchunk,
                                                      double *__restrict__ part, int nsplit)
{
    constexpr int BS = 64 * NW;
    __shared__ double2 lds[2][TILE * 5];
    int ib, split;
    eval_block_coords(nsplit, ib, split);
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int ibase = ib * (BS * IPL);
    I64 b[IPL];
    int lo, hi;
    bool bad;
    load_i_f64<IPL, BS>(A.jrec, idx, n_act, ibase, 0, n, b, lo, hi, bad);
    if (bad)
        raise_err(A.status, kErrIndex);
    tiles_f64<IPL, NW, TILE>(A.jrec, jbeg, jend, b, lo, hi, eps2, lds);
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + (int)threadIdx.x;
        if (slot < n_act) {
#pragma unroll
            for (int c = 0; c < 10; ++c)
                part[((size_t)split * 10 + c) * n_act + slot] = b[q].acc[c];
        }
    }
}

// ------------------------------------------------------ pairwise (split) ----
// Same decomposition with the split-precision interaction (tiles_split).
template <int IPL, int NW, int TILE>
__global__ __launch_bounds__(64 * NW) void k_eval_split(Arrays A, int n, const int32_t *__restrict__ idx,
                                                        int n_act, float eps2, int jchunk,
                                                        double *__restrict__ part, int nsplit)
{
    constexpr int BS = 64 * NW;
    __shared__ float4 lds[2][TILE * 4];
    int ib, split;
    eval_block_coords(nsplit, ib, split);
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int ibase = ib * (BS * IPL);
    I32 b[IPL];
    int lo, hi;
    bool bad;
    load_i_split<IPL, BS>(A.jrec32, idx, n_act, ibase, 0, n, b, lo, hi, bad);
    if (bad)
        raise_err(A.status, kErrIndex);
    tiles_split<IPL, NW, TILE>(A.jrec32, jbeg, jend, b, lo, hi, eps2, lds);
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + (int)threadIdx.x;
        if (slot < n_act) {
#pragma unroll
            for (int c = 0; c < 10; ++c)
                part[((size_t)split * 10 + c) * n_act + slot] = b[q].acc[c];
        }
    }
}

// --------------------------------------------- small active sets (FP64) ----
// A one-wave workgroup holds P = 64 / W active bodies with W lanes each: lane w of a
// body takes records w, w + W, ... of the workgroup's j-range, staged through LDS
// tiles of 64 records or, for DIRECT, read straight from memory (a few records per
// lane, where a tile would not hide the load latency). The W lane sums of a body are
// combined by a fixed butterfly and written as the split's partial sums, so a wave
// stays full for the one to a few dozen active bodies of a sparse block step.
template <bool DIRECT>
__global__ __launch_bounds__(64) void k_eval_lanes_f64(Arrays A, int n, const int32_t *__restrict__ idx,
                                                       int n_act, double eps2, int lw, int jchunk,
                                                       double *__restrict__ part, int nsplit)
{
    __shared__ double2 lds[DIRECT ? 1 : 2][kLaneTile * 5];
    int g, split;
    eval_block_coords(nsplit, g, split);
    const int W = 1 << lw, w = (int)threadIdx.x & (W - 1);
    const int slot = (g << (6 - lw)) + ((int)threadIdx.x >> lw);
    const double2 *__restrict__ src = reinterpret_cast<const double2 *>(A.jrec);
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    // a direct sweep's first records are requested before the active body's record
    DirectHead head{};
    if constexpr (DIRECT)
        head = direct_head(src, jbeg, jend, W, w);
    int i = idx[slot < n_act ? slot : n_act - 1];
    if ((unsigned)i >= (unsigned)n) {
        raise_err(A.status, kErrIndex);
        i = 0;
    }
    I64 b;
    {
        const double2 *r = src + (size_t)i * 5;
        const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
        b.x[0] = r0.x; b.x[1] = r0.y; b.x[2] = r1.x;
        b.v[0] = r1.y; b.v[1] = r2.x; b.v[2] = r2.y;
        b.a[0] = r3.x; b.a[1] = r3.y; b.a[2] = r4.x;
#pragma unroll
        for (int c = 0; c < 10; ++c)
            b.acc[c] = 0.0;
        b.self = i;
    }
    const int lo = wave_min_i32(i), hi = wave_max_i32(i);
    if constexpr (DIRECT)
        sweep_direct_f64(src, jbeg, jend, W, w, b, lo, hi, eps2, head);
    else
        sweep_lds_f64(src, jbeg, jend, W, lw, w, b, lo, hi, eps2, lds);
#pragma unroll
    for (int c = 0; c < 10; ++c)
        b.acc[c] = lane_butterfly(b.acc[c], W);
    if (w == 0 && slot < n_act) {
#pragma unroll
        for (int c = 0; c < 10; ++c)
            part[((size_t)split * 10 + c) * n_act + slot] = b.acc[c];
    }
}

// Sum over the S j-splits, out[e] = sum_s part[s][e], in a fixed order: G threads
// share an element, thread g adds s = g, g + G, ... in turn (four independent
// chains, combined in a fixed pattern), then the G results are combined by a fixed
// tree in LDS. G grows with S so that a large S is not one long chain of
// dependent loads; for a given (S, count) the order is always the same.
template <int G>
__global__ __launch_bounds__(256) void k_reduce_splits(const double *__restrict__ part, int S,
                                                       int64_t count, double *__restrict__ dst,
                                                       double *__restrict__ dst2)
{
    constexpr int E = 256 / G;  // elements per workgroup
    __shared__ double red[256];
    const int el = threadIdx.x % E, g = threadIdx.x / E;
    const int64_t e = (int64_t)blockIdx.x * E + el;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (e < count) {
        int s = g;
        for (; s + 3 * G < S; s += 4 * G) {
            a0 += part[(size_t)s * count + e];
            a1 += part[(size_t)(s + G) * count + e];
            a2 += part[(size_t)(s + 2 * G) * count + e];
            a3 += part[(size_t)(s + 3 * G) * count + e];
        }
        for (; s < S; s += G)
            a0 += part[(size_t)s * count + e];
    }
    double acc = (a0 + a1) + (a2 + a3);
    if (G > 1) {
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = G / 2; w > 0; w >>= 1) {
            if (g < w)
                red[threadIdx.x] += red[threadIdx.x + w * E];
            __syncthreads();
        }
        acc = red[threadIdx.x];
    }
    if (g == 0 && e < count) {
        dst[e] = acc;
        if (dst2)
            dst2[e] = acc;
    }
}

// ---------------------------------------------------------------- corrector ----
// Hermite-6 corrector of the active bodies (correct_body) to the block time.
__global__ __launch_bounds__(256) void k_correct(Arrays A, int n, const int32_t *__restrict__ idx,
                                                 int n_act, int64_t tick, double tick_size)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_act)
        return;
    const int i = idx[q];
    // a body listed twice would be corrected twice: the list must be strictly ascending
    if ((unsigned)i >= (unsigned)n || (q > 0 && idx[q - 1] >= i)) {
        raise_err(A.status, kErrIndex);
        return;
    }
    const int64_t ti = A.tick[i];
    if (ti >= tick) {
        raise_err(A.status, kErrLevel);
        return;
    }
    const double h = (double)(tick - ti) * tick_size;
    const bool finite = correct_body(A.x, A.v, A.a, A.j, A.s, A.c, A.a4n, A.a5n, (size_t)n,
                                     (size_t)i, A.evalbuf + q, (size_t)n_act, h);
    A.phi[i] = A.evalbuf[(size_t)9 * n_act + q];
    A.tick[i] = tick;
    if (!finite)
        raise_err(A.status, kErrNumeric);
}

// -------------------------------------------------------------- step levels ----
// New levels of the given bodies (level_for_body).
__global__ __launch_bounds__(256) void k_timesteps(Arrays A, int n, const int32_t *__restrict__ idx,
                                                   int n_act, int init, double eta, double eta_init,
                                                   int dt_max_log2, int L)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_act)
        return;
    const int i = idx[q];
    if ((unsigned)i >= (unsigned)n) {
        raise_err(A.status, kErrIndex);
        return;
    }
    bool dtmin;
    A.level[i] = level_for_body(A.a, A.j, A.s, A.c, A.a4n, A.a5n, (size_t)n, (size_t)i, A.tick[i],
                                A.level[i], init, eta, eta_init, dt_max_log2, L, &dtmin);
    if (dtmin)
        raise_err(A.status, kErrDtMin);
}

// --------------------------------------------------------------- active set ----
// tick_next = min_i (t_i + dt_i); active = {i : t_i + dt_i == tick_next}, ascending.
// Three passes over kActChunk-body chunks: chunk minima, then per-chunk counts
// against the global minimum, then a scatter at each chunk's exclusive offset with
// an in-chunk ballot scan (so the list comes out in ascending order).
__device__ __forceinline__ int64_t body_end(const Arrays &A, int i, int L)
{
    int lv = A.level[i];
    if (lv < 0 || lv > L) {
        raise_err(A.status, kErrLevel);
        lv = L;
    }
    return A.tick[i] + ((int64_t)1 << (L - lv));
}

__global__ __launch_bounds__(kActBS) void k_act_min(Arrays A, int n, int L)
{
    __shared__ int64_t red[kActBS / 64];
    const int base = blockIdx.x * kActChunk;
    int64_t mn = INT64_MAX;
#pragma unroll
    for (int r = 0; r < kActPerThread; ++r) {
        const int i = base + r * kActBS + threadIdx.x;
        if (i < n) {
            const int64_t e = body_end(A, i, L);
            mn = e < mn ? e : mn;
        }
    }
    mn = wave_min_i64(mn);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = red[0];
        for (int w = 1; w < kActBS / 64; ++w)
            m = red[w] < m ? red[w] : m;
        A.act_bmin[blockIdx.x] = m;
    }
}

__device__ int64_t block_global_min(const Arrays &A, int nb, int64_t *red)
{
    int64_t mn = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kActBS) {
        const int64_t v = A.act_bmin[b];
        mn = v < mn ? v : mn;
    }
    mn = wave_min_i64(mn);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = mn;
    __syncthreads();
    int64_t m = red[0];
    for (int w = 1; w < kActBS / 64; ++w)
        m = red[w] < m ? red[w] : m;
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(kActBS) void k_act_count(Arrays A, int n, int L, int nb)
{
    __shared__ int64_t red[kActBS / 64];
    __shared__ int cnt[kActBS / 64];
    const int64_t tn = block_global_min(A, nb, red);
    const int base = blockIdx.x * kActChunk;
    int c = 0;
#pragma unroll
    for (int r = 0; r < kActPerThread; ++r) {
        const int i = base + r * kActBS + threadIdx.x;
        if (i < n && body_end(A, i, L) == tn)
            ++c;
    }
    c = wave_sum_i32(c);
    if ((threadIdx.x & 63) == 0)
        cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kActBS / 64; ++w)
            t += cnt[w];
        A.act_bcnt[blockIdx.x] = t;
        if (blockIdx.x == 0)
            A.status->tick_next = tn;
    }
}

__global__ __launch_bounds__(kActBS) void k_act_scatter(Arrays A, int n, int L, int nb,
                                                        int32_t *__restrict__ out)
{
    __shared__ int red[kActBS / 64];
    __shared__ int wcnt[kActBS / 64];
    const int64_t tn = A.status->tick_next;
    // exclusive offset of this chunk (and, in block 0, the total)
    int off = 0, tot = 0;
    for (int b = threadIdx.x; b < nb; b += kActBS) {
        const int v = A.act_bcnt[b];
        if (b < (int)blockIdx.x)
            off += v;
        tot += v;
    }
    off = wave_sum_i32(off);
    tot = wave_sum_i32(tot);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = off;
    __syncthreads();
    int base_off = 0;
    for (int w = 0; w < kActBS / 64; ++w)
        base_off += red[w];
    __syncthreads();
    if (blockIdx.x == 0) {
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kActBS / 64; ++w)
                t += red[w];
            A.status->n_act = t;
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blockIdx.x * kActChunk;
    for (int r = 0; r < kActPerThread; ++r) {
        const int i = base + r * kActBS + threadIdx.x;
        const bool act = (i < n) && body_end(A, i, L) == tn;
        const unsigned long long mask = __ballot(act);
        if (lane == 0)
            wcnt[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, round_tot = 0;
        for (int w = 0; w < kActBS / 64; ++w) {
            before += (w < wave) ? wcnt[w] : 0;
            round_tot += wcnt[w];
        }
        if (act) {
            const int pos = base_off + before + __popcll(mask & ((1ull << lane) - 1ull));
            out[pos] = i;
        }
        base_off += round_tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------------- energy ----
// E_kin = sum m v^2 / 2 over the predicted velocities and
// E_pot = -1/2 sum_i m_i sum_{j != i} m_j / sqrt(r^2 + eps^2), from the j-records.
// Potential per body with j-splits (partials per split), then fixed-order sums.
template <int TILE>
__global__ __launch_bounds__(kEnBS) void k_potential(Arrays A, int n, double eps2, int jchunk,
                                                     double *__restrict__ part)
{
    constexpr int BS = kEnBS;
    constexpr int CH = TILE * 5;
    static_assert(CH % BS == 0, "tile chunks must split evenly over the workgroup");
    constexpr int CPT = CH / BS;
    __shared__ double2 lds[CH];
    const int tid = threadIdx.x;
    const int split = blockIdx.y;
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int i0 = blockIdx.x * BS;
    const int i = min(i0 + tid, n - 1);
    const double2 *src = reinterpret_cast<const double2 *>(A.jrec);
    const double xi = A.jrec[(size_t)i * kRecD + 0], yi = A.jrec[(size_t)i * kRecD + 1],
                 zi = A.jrec[(size_t)i * kRecD + 2];
    const int ilo = i0, ihi = min(i0 + BS, n) - 1;
    double phi = 0.0;
    for (int j0 = jbeg; j0 < jend; j0 += TILE) {
        const int valid = (jend - j0) * 5;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = c * BS + tid;
            double2 v;
            if (ch < valid)
                v = src[(size_t)j0 * 5 + ch];
            else
                v = (ch % 5) == 0 ? make_double2(kFar, kFar)
                  : (ch % 5) == 1 ? make_double2(kFar, 0.0)
                                  : make_double2(0.0, 0.0);
            lds[ch] = v;
        }
        __syncthreads();
        const bool masked = !(ihi < j0 || ilo >= j0 + TILE);
        for (int jj = 0; jj < TILE; ++jj) {
            const double2 p0 = lds[jj * 5 + 0], p1 = lds[jj * 5 + 1], p4 = lds[jj * 5 + 4];
            const double dx = p0.x - xi, dy = p0.y - yi, dz = p1.x - zi;
            double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double mj = p4.y;
            if (masked && j0 + jj == i) {
                mj = 0.0;
                r2 = 1.0;
            }
            phi = __builtin_fma(mj, rsqrt_f64(r2), phi);
        }
        __syncthreads();
    }
    if (i0 + tid < n)
        part[(size_t)split * n + i0 + tid] = phi;
}

__global__ __launch_bounds__(kEnBS) void k_energy_blocks(Arrays A, int n, int S,
                                                         const double *__restrict__ part)
{
    __shared__ double rk[kEnBS], rp[kEnBS];
    const int i = blockIdx.x * kEnBS + threadIdx.x;
    double ek = 0.0, ep = 0.0;
    if (i < n) {
        double phi = part[i];
        for (int s = 1; s < S; ++s)
            phi += part[(size_t)s * n + i];
        const double *r = A.jrec + (size_t)i * kRecD;
        const double m = r[9];
        const double vx = r[3], vy = r[4], vz = r[5];
        ek = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        ep = -0.5 * m * phi;
    }
    rk[threadIdx.x] = ek;
    rp[threadIdx.x] = ep;
    __syncthreads();
    for (int w = kEnBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rk[threadIdx.x] += rk[threadIdx.x + w];
            rp[threadIdx.x] += rp[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A.en_bsum[2 * blockIdx.x + 0] = rk[0];
        A.en_bsum[2 * blockIdx.x + 1] = rp[0];
    }
}

__global__ __launch_bounds__(64) void k_energy_final(Arrays A, int nb)
{
    if (threadIdx.x == 0) {
        double ek = 0.0, ep = 0.0;
        for (int b = 0; b < nb; ++b) {
            ek += A.en_bsum[2 * b + 0];
            ep += A.en_bsum[2 * b + 1];
        }
        A.status->ekin = ek;
        A.status->epot = ep;
    }
}

unsigned blocks_for(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace

// ================================================================= launchers ====
hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t st) { return fill(p, v, count, st); }
hipError_t launch_fill_i64(int64_t *p, int64_t v, size_t count, hipStream_t st) { return fill(p, v, count, st); }
hipError_t launch_fill_i32(int32_t *p, int32_t v, size_t count, hipStream_t st) { return fill(p, v, count, st); }

hipError_t launch_iota(int32_t *p, int64_t count, hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(count, 256)), dim3(256), 0, st, p, (int)count);
    return hipGetLastError();
}

int act_blocks(int64_t n) { return (int)((n + kActChunk - 1) / kActChunk); }
int en_blocks(int64_t n) { return (int)((n + kEnBS - 1) / kEnBS); }

hipError_t launch_predict(const Arrays &A, int64_t n, int64_t tick, int dt_min_log2, bool split,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_predict, dim3(blocks_for(n, 256)), dim3(256), 0, st, A, (int)n, tick,
                       ldexp(1.0, dt_min_log2), (int)split);
    return hipGetLastError();
}

hipError_t launch_get_predicted(const Arrays &A, int64_t n, double *xp, double *vp, double *ap,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_get_predicted, dim3(blocks_for(n, 256)), dim3(256), 0, st, A.jrec, (int)n,
                       xp, vp, ap);
    return hipGetLastError();
}

hipError_t launch_pack_records(const double *m, const double *xp, const double *vp,
                               const double *ap, int64_t n, double *jrec, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_records, dim3(blocks_for(n, 256)), dim3(256), 0, st, m, xp, vp, ap,
                       (int)n, jrec);
    return hipGetLastError();
}

hipError_t launch_poison_on_index_error(const Status *stt, double *out, int64_t count,
                                        hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(k_poison_on_index_error, dim3((unsigned)blocks), dim3(256), 0, st, stt, out,
                       count);
    return hipGetLastError();
}

hipError_t launch_copy_acc_to_jrec(const Arrays &A, int64_t n, bool split, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_acc_to_jrec, dim3(blocks_for(n, 256)), dim3(256), 0, st, A, (int)n,
                       (int)split);
    return hipGetLastError();
}

hipError_t launch_start_store(const Arrays &A, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_start_store, dim3(blocks_for(n, 256)), dim3(256), 0, st, A, (int)n);
    return hipGetLastError();
}

template <int IPL, int NW, int TILE>
static hipError_t run_eval(const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                           int64_t n_act, double eps, bool split, double *dst, hipStream_t st)
{
    // XCD-aware 1-D grid when the splits divide evenly over the eight XCDs
    const bool xcd = P.splits > 1 && (P.splits % 8) == 0;
    const dim3 grid = xcd ? dim3(P.iblocks * P.splits, 1) : dim3(P.iblocks, P.splits);
    const dim3 block(64 * NW);
    if (split)
        hipLaunchKernelGGL((k_eval_split<IPL, NW, TILE>), grid, block, 0, st, A, (int)n, idx,
                           (int)n_act, (float)(eps * eps), P.jchunk, dst, P.splits);
    else
        hipLaunchKernelGGL((k_eval_f64<IPL, NW, TILE>), grid, block, 0, st, A, (int)n, idx,
                           (int)n_act, eps * eps, P.jchunk, dst, P.splits);
    return hipGetLastError();
}

hipError_t launch_eval(const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                       int64_t n_act, double eps, bool split, double *out, hipStream_t st)
{
    if (n_act <= 0)
        return hipSuccess;
    double *dst = (P.splits == 1) ? A.evalbuf : A.part;
    hipError_t e;
#define NB_SHAPE(I, W, T)                                                                  \
    else if (P.ipl == I && P.waves == W && P.tile == T) e =                                \
        run_eval<I, W, T>(A, P, n, idx, n_act, eps, split, dst, st);
    if (P.lw >= 0 && P.waves > 1) {
        // group kernel: one launch when it reduces the splits itself
        if (split)
            return hipErrorInvalidValue;
        if (P.splits == 1 || P.fused)
            return launch_eval_group(A, P, n, idx, n_act, eps, P.fused ? A.ectr : nullptr,
                                     A.evalbuf, out, st);
        e = launch_eval_group(A, P, n, idx, n_act, eps, nullptr, A.evalbuf, out, st);
    } else if (P.lw >= 0) {
        if (split)
            return hipErrorInvalidValue;
        const bool xcd = P.splits > 1 && (P.splits % 8) == 0;
        const dim3 grid = xcd ? dim3(P.iblocks * P.splits, 1) : dim3(P.iblocks, P.splits);
        if (P.tile == 0)
            hipLaunchKernelGGL(k_eval_lanes_f64<true>, grid, dim3(64), 0, st, A, (int)n, idx,
                               (int)n_act, eps * eps, P.lw, P.jchunk, dst, P.splits);
        else
            hipLaunchKernelGGL(k_eval_lanes_f64<false>, grid, dim3(64), 0, st, A, (int)n, idx,
                               (int)n_act, eps * eps, P.lw, P.jchunk, dst, P.splits);
        e = hipGetLastError();
    }
    NB_SHAPE(1, 1, 64) NB_SHAPE(1, 1, 128) NB_SHAPE(1, 2, 128) NB_SHAPE(1, 1, 256)
    NB_SHAPE(1, 2, 256) NB_SHAPE(1, 4, 256) NB_SHAPE(2, 1, 64) NB_SHAPE(2, 1, 128)
    NB_SHAPE(2, 2, 128) NB_SHAPE(2, 1, 256) NB_SHAPE(2, 2, 256) NB_SHAPE(2, 4, 256)
    else return hipErrorInvalidValue;
#undef NB_SHAPE
    if (e != hipSuccess)
        return e;
    const int64_t count = 10 * n_act;
    if (P.splits > 1) {
        const double *pp = A.part;
        if (P.splits <= 16)
            hipLaunchKernelGGL(k_reduce_splits<1>, dim3(blocks_for(count, 256)), dim3(256), 0, st,
                               pp, P.splits, count, A.evalbuf, out);
        else if (P.splits <= 128)
            hipLaunchKernelGGL(k_reduce_splits<8>, dim3(blocks_for(count, 32)), dim3(256), 0, st,
                               pp, P.splits, count, A.evalbuf, out);
        else
            hipLaunchKernelGGL(k_reduce_splits<64>, dim3(blocks_for(count, 4)), dim3(256), 0, st,
                               pp, P.splits, count, A.evalbuf, out);
        return hipGetLastError();
    }
    if (out)
        return hipMemcpyAsync(out, A.evalbuf, sizeof(double) * count, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
}

hipError_t launch_correct(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act, int64_t tick,
                          int dt_min_log2, hipStream_t st)
{
    if (n_act <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_correct, dim3(blocks_for(n_act, 256)), dim3(256), 0, st, A, (int)n, idx,
                       (int)n_act, tick, ldexp(1.0, dt_min_log2));
    return hipGetLastError();
}

hipError_t launch_timesteps(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act, int init,
                            double eta, double eta_init, int dt_max_log2, int dt_min_log2,
                            hipStream_t st)
{
    if (n_act <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_timesteps, dim3(blocks_for(n_act, 256)), dim3(256), 0, st, A, (int)n, idx,
                       (int)n_act, init, eta, eta_init, dt_max_log2, dt_max_log2 - dt_min_log2);
    return hipGetLastError();
}

hipError_t launch_active(const Arrays &A, int64_t n, int L, int32_t *idx_out, hipStream_t st)
{
    const int nb = act_blocks(n);
    hipLaunchKernelGGL(k_act_min, dim3(nb), dim3(kActBS), 0, st, A, (int)n, L);
    hipLaunchKernelGGL(k_act_count, dim3(nb), dim3(kActBS), 0, st, A, (int)n, L, nb);
    hipLaunchKernelGGL(k_act_scatter, dim3(nb), dim3(kActBS), 0, st, A, (int)n, L, nb, idx_out);
    return hipGetLastError();
}

hipError_t launch_energy(const Arrays &A, int64_t n, double eps, int64_t partial_slots, hipStream_t st)
{
    constexpr int TILE = 256;
    const int ib = en_blocks(n);
    // j-splits so that the potential pass has a few thousand waves
    int64_t S = (8192 + 4 * (int64_t)ib - 1) / (4 * (int64_t)ib);
    const int64_t max_tiles = (n + TILE - 1) / TILE;
    if (S > max_tiles) S = max_tiles;
    const int64_t cap = (10 * partial_slots) / n;
    if (S > cap) S = cap;
    if (S < 1) S = 1;
    int64_t per = (n + S - 1) / S;
    per = (per + TILE - 1) / TILE * TILE;
    const int splits = (int)((n + per - 1) / per);
    hipLaunchKernelGGL(k_potential<TILE>, dim3(ib, splits), dim3(kEnBS), 0, st, A, (int)n, eps * eps,
                       (int)per, A.part);
    hipLaunchKernelGGL(k_energy_blocks, dim3(ib), dim3(kEnBS), 0, st, A, (int)n, splits,
                       (const double *)A.part);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, st, A, ib);
    return hipGetLastError();
}

}  // namespace nb
