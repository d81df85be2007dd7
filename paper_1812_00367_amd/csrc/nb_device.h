// nb_device.h -- device functions shared by the single-system kernels
// (nbody_kernels.hip) and the batched kernels (nbody_batch.hip): the pairwise
// interaction in FP64 and split precision with its LDS tile loop, and the per-body
// predictor, corrector and step-level rules. Formulas: 6th-order Hermite scheme
// (Nitadori & Makino 2008) as named by the paper's section "Code implementation";
// each function states the ones it uses.
#pragma once

#include "nb_internal.h"
#include "nb_math.h"

#include <math.h>

namespace nb {


// ------------------------------------------------------------ wave reductions ----
__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup -> (active-body block, j-split). Workgroups are dispatched to the eight
// XCDs round-robin (workgroup l on XCD l % 8), each XCD with its own L2. When S is a
// multiple of 8, a 1-D grid is launched and XCD x is given the contiguous splits
// [x S/8, (x+1) S/8), so each XCD's L2 fetches only its eighth of the j-stream.
__device__ __forceinline__ void eval_block_coords(int nsplit, int &ib, int &split)
{
    if (gridDim.y == 1 && nsplit > 1) {
        const int l = blockIdx.x, x = l & 7, k = l >> 3, sx = nsplit >> 3;
        split = x * sx + k % sx;
        ib = k / sx;
    } else {
        ib = blockIdx.x;
        split = blockIdx.y;
    }
}

// Whether any lane of the wave holds an own body with index in [j0, j0 + len): the
// self pair is masked only on such tiles (wave-uniform decision).
template <typename B, int IPL>
__device__ __forceinline__ bool wave_has_self(const B (&b)[IPL], int j0, int len)
{
    bool mine = false;
#pragma unroll
    for (int q = 0; q < IPL; ++q)
        mine |= (unsigned)(b[q].self - j0) < (unsigned)len;
    return __ballot(mine) != 0;
}

// --------------------------------------------------------- pairwise (FP64) ----
// For an active body i and every j != i (predicted quantities; softening eps):
//   r = x_j - x_i, v = v_j - v_i, a = a_j - a_i, R = r.r + eps^2,
//   m3 = m_j R^(-3/2), alpha = r.v / R, beta = (v.v + r.a) / R + alpha^2,
//   A = m3 r, J = m3 v - 3 alpha A, S = m3 a - 6 alpha J - 3 beta A, phi -= m_j R^(-1/2).
// They are accumulated in the equivalent fused form J = m3 w with w = v - 3 alpha r and
// S = m3 u with u = a - 3 beta r - 6 alpha w, so every accumulation is one FMA.
struct I64 {
    double x[3], v[3], a[3];
    double acc[10];
    int self;
};

template <bool MASK>
__device__ __forceinline__ void interact_f64(I64 &b, const double2 p0, const double2 p1,
                                             const double2 p2, const double2 p3, const double2 p4,
                                             double eps2, int jglob)
{
    const double dx = p0.x - b.x[0], dy = p0.y - b.x[1], dz = p1.x - b.x[2];
    const double dvx = p1.y - b.v[0], dvy = p2.x - b.v[1], dvz = p2.y - b.v[2];
    const double dax = p3.x - b.a[0], day = p3.y - b.a[1], daz = p4.x - b.a[2];
    double mj = p4.y;
    double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
    if (MASK) {
        const bool self = (jglob == b.self);
        mj = self ? 0.0 : mj;
        r2 = self ? 1.0 : r2;
    }
    const double rv = __builtin_fma(dx, dvx, __builtin_fma(dy, dvy, dz * dvz));
    const double vvra = __builtin_fma(
        dvx, dvx,
        __builtin_fma(dvy, dvy,
                      __builtin_fma(dvz, dvz, __builtin_fma(dx, dax, __builtin_fma(dy, day, dz * daz)))));
    const double rinv = rsqrt_f64(r2);
    const double rinv2 = rinv * rinv;
    const double alpha = rv * rinv2;
    const double beta = __builtin_fma(alpha, alpha, vvra * rinv2);
    const double mr = mj * rinv;
    const double m3 = mr * rinv2;
    const double a3 = 3.0 * alpha;
    const double a6 = 6.0 * alpha;
    const double b3 = 3.0 * beta;
    b.acc[0] = __builtin_fma(m3, dx, b.acc[0]);
    b.acc[1] = __builtin_fma(m3, dy, b.acc[1]);
    b.acc[2] = __builtin_fma(m3, dz, b.acc[2]);
    const double wx = __builtin_fma(-a3, dx, dvx);
    const double wy = __builtin_fma(-a3, dy, dvy);
    const double wz = __builtin_fma(-a3, dz, dvz);
    b.acc[3] = __builtin_fma(m3, wx, b.acc[3]);
    b.acc[4] = __builtin_fma(m3, wy, b.acc[4]);
    b.acc[5] = __builtin_fma(m3, wz, b.acc[5]);
    const double ux = __builtin_fma(-a6, wx, __builtin_fma(-b3, dx, dax));
    const double uy = __builtin_fma(-a6, wy, __builtin_fma(-b3, dy, day));
    const double uz = __builtin_fma(-a6, wz, __builtin_fma(-b3, dz, daz));
    b.acc[6] = __builtin_fma(m3, ux, b.acc[6]);
    b.acc[7] = __builtin_fma(m3, uy, b.acc[7]);
    b.acc[8] = __builtin_fma(m3, uz, b.acc[8]);
    b.acc[9] -= mr;
}

// IPL active bodies per lane from the list act[0, n_act): slot ibase + q*BS + tid
// (slots past the end repeat the last entry and are not written back). Indices
// outside [idx_lo, idx_hi) are replaced by idx_lo and reported through *bad.
// lo/hi return the wave's smallest and largest own index (for self masking).
template <int IPL, int BS>
__device__ __forceinline__ void load_i_f64(const double *__restrict__ jrec,
                                           const int32_t *__restrict__ act, int n_act, int ibase,
                                           int idx_lo, int idx_hi, I64 (&b)[IPL], int &lo, int &hi,
                                           bool &bad)
{
    lo = 0x7fffffff;
    hi = -1;
    bad = false;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + (int)threadIdx.x;
        int i = act[slot < n_act ? slot : n_act - 1];
        if (i < idx_lo || i >= idx_hi) {
            bad = true;
            i = idx_lo;
        }
        b[q].self = i;
        const double2 *r = reinterpret_cast<const double2 *>(jrec + (size_t)i * kRecD);
        const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
        b[q].x[0] = r0.x; b[q].x[1] = r0.y; b[q].x[2] = r1.x;
        b[q].v[0] = r1.y; b[q].v[1] = r2.x; b[q].v[2] = r2.y;
        b[q].a[0] = r3.x; b[q].a[1] = r3.y; b[q].a[2] = r4.x;
#pragma unroll
        for (int c = 0; c < 10; ++c)
            b[q].acc[c] = 0.0;
        lo = min(lo, i);
        hi = max(hi, i);
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
}

// Sweep the j-records [jbeg, jend) tile by tile through LDS (lds: two buffers of
// TILE records), double-buffered with register staging: every thread issues its
// 16-byte loads unconditionally (an out-of-range chunk reloads chunk 0) so they
// stay in flight during the previous tile's arithmetic, and padding records
// {far, far, far, 0 ..., m = 0} are substituted when storing to LDS. The self pair
// is masked only on tiles that contain one of the wave's own indices [lo, hi].
// Every thread of the workgroup must call this (it synchronises).
template <int IPL, int NW, int TILE>
__device__ __forceinline__ void tiles_f64(const double *__restrict__ jrec, int jbeg, int jend,
                                          I64 (&b)[IPL], int lo, int hi, double eps2,
                                          double2 (*lds)[TILE * 5])
{
    constexpr int BS = 64 * NW;
    constexpr int CH = TILE * 5;  // 16-byte chunks per tile
    static_assert(CH % BS == 0, "tile chunks must split evenly over the workgroup");
    constexpr int CPT = CH / BS;
    const int tid = threadIdx.x;
    const double2 *__restrict__ src = reinterpret_cast<const double2 *>(jrec);
    const int ntiles = (jend - jbeg + TILE - 1) / TILE;
    double2 stage[CPT];
    int valid = 0;
    auto gload = [&](int t) {
        const int j0 = jbeg + t * TILE;
        valid = (jend - j0) * 5;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = c * BS + tid;
            stage[c] = src[ch < valid ? (size_t)j0 * 5 + ch : 0];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = c * BS + tid;
            const bool ok = ch < valid;
            const int part5 = ch % 5;
            double2 v;
            v.x = ok ? stage[c].x : (part5 <= 1 ? kFar : 0.0);
            v.y = ok ? stage[c].y : (part5 == 0 ? kFar : 0.0);
            lds[buf][ch] = v;
        }
    };
    if (ntiles > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles)
            gload(t + 1);
        const int j0 = jbeg + t * TILE;
        const double2 *L = lds[buf];
        if ((hi < j0 || lo >= j0 + TILE) || !wave_has_self(b, j0, TILE)) {
            // the next record's LDS reads are issued before this record's arithmetic
            double2 p0 = L[0], p1 = L[1], p2 = L[2], p3 = L[3], p4 = L[4];
#pragma unroll 2
            for (int jj = 0; jj < TILE; ++jj) {
                const int nx = (jj + 1 < TILE ? jj + 1 : jj) * 5;
                const double2 n0 = L[nx + 0], n1 = L[nx + 1], n2 = L[nx + 2], n3 = L[nx + 3],
                              n4 = L[nx + 4];
#pragma unroll
                for (int q = 0; q < IPL; ++q)
                    interact_f64<false>(b[q], p0, p1, p2, p3, p4, eps2, 0);
                p0 = n0; p1 = n1; p2 = n2; p3 = n3; p4 = n4;
            }
        } else {
            for (int jj = 0; jj < TILE; ++jj) {
                const double2 p0 = L[jj * 5 + 0], p1 = L[jj * 5 + 1], p2 = L[jj * 5 + 2],
                              p3 = L[jj * 5 + 3], p4 = L[jj * 5 + 4];
#pragma unroll
                for (int q = 0; q < IPL; ++q)
                    interact_f64<true>(b[q], p0, p1, p2, p3, p4, eps2, j0 + jj);
            }
        }
        if (t + 1 < ntiles)
            lstore(buf ^ 1);
        __syncthreads();
    }
}

// ------------------------------------------- W lanes per active body (FP64) ----
// Small active sets: W lanes (a power of two) share one active body, lane w of a body
// taking records w, w + W, ... of a j-range; the W partial sums of a body are then
// combined by a fixed butterfly, so the result depends only on W and the range.
constexpr int kLaneStageD = kLaneTile * 5 / 64;  // 16-byte chunks per lane per tile

template <typename T>
__device__ __forceinline__ T lane_butterfly(T v, int W)
{
    for (int o = W >> 1; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

struct Rec64 {
    double2 p0, p1, p2, p3, p4;
};

__device__ __forceinline__ Rec64 load_rec64(const double2 *__restrict__ src, int j)
{
    const double2 *r = src + (size_t)j * 5;
    return Rec64{r[0], r[1], r[2], r[3], r[4]};
}

// Rounds k = 0, 1, ...: lane w takes record jbeg + k W + w. Loads run two rounds
// ahead. A record past jend is replaced by jbeg's and masked like the self pair (its
// index set to the lane's own body); masking is used only on rounds that hold the
// wave's own bodies or the end of the range. The first two rounds' records (the
// head) can be requested early, before the active body's own record is loaded.
struct DirectHead {
    Rec64 c, nx;
};

__device__ __forceinline__ DirectHead direct_head(const double2 *__restrict__ src, int jbeg, int jend,
                                                  int W, int w)
{
    const int rounds = (jend - jbeg + W - 1) / W;
    auto at = [&](int k) { const int j = jbeg + k * W + w; return j < jend ? j : jbeg; };
    return DirectHead{load_rec64(src, at(0)), load_rec64(src, at(rounds > 1 ? 1 : 0))};
}

__device__ __forceinline__ void sweep_direct_f64(const double2 *__restrict__ src, int jbeg, int jend,
                                                 int W, int w, I64 &b, int lo, int hi, double eps2,
                                                 DirectHead h)
{
    const I64(&one)[1] = reinterpret_cast<const I64(&)[1]>(b);
    const int rounds = (jend - jbeg + W - 1) / W;
    auto idx = [&](int k) { return jbeg + k * W + w; };
    auto at = [&](int k) { const int j = idx(k); return j < jend ? j : jbeg; };
    Rec64 c = h.c;
    Rec64 nx = h.nx;
    for (int k = 0; k < rounds; ++k) {
        const Rec64 f = load_rec64(src, at(k + 2 < rounds ? k + 2 : k));
        const int r0 = jbeg + k * W;
        if (r0 + W <= jend && ((hi < r0 || lo >= r0 + W) || !wave_has_self(one, r0, W))) {
            interact_f64<false>(b, c.p0, c.p1, c.p2, c.p3, c.p4, eps2, 0);
        } else {
            const int j = idx(k);
            interact_f64<true>(b, c.p0, c.p1, c.p2, c.p3, c.p4, eps2, j < jend ? j : b.self);
        }
        c = nx;
        nx = f;
    }
}

__device__ __forceinline__ void sweep_direct_f64(const double2 *__restrict__ src, int jbeg, int jend,
                                                 int W, int w, I64 &b, int lo, int hi, double eps2)
{
    sweep_direct_f64(src, jbeg, jend, W, w, b, lo, hi, eps2, direct_head(src, jbeg, jend, W, w));
}

// LDS tiles of 64 records, double-buffered through registers (as the single-system
// kernel): lane w reads records w, w + W, ... of each tile.
__device__ __forceinline__ void sweep_lds_f64(const double2 *__restrict__ src, int jbeg, int jend,
                                              int W, int lw, int w, I64 &b, int lo, int hi, double eps2,
                                              double2 (*lds)[kLaneTile * 5])
{
    const int lane = threadIdx.x;
    const int ntiles = (jend - jbeg + kLaneTile - 1) / kLaneTile;
    double2 stage[kLaneStageD];
    int valid = 0;
    auto gload = [&](int t) {
        const int j0 = jbeg + t * kLaneTile;
        valid = (jend - j0) * 5;
#pragma unroll
        for (int c = 0; c < kLaneStageD; ++c) {
            const int ch = c * 64 + lane;
            stage[c] = src[ch < valid ? (size_t)j0 * 5 + ch : 0];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < kLaneStageD; ++c) {
            const int ch = c * 64 + lane;
            const bool ok = ch < valid;
            const int part5 = ch % 5;
            double2 v;
            v.x = ok ? stage[c].x : (part5 <= 1 ? kFar : 0.0);
            v.y = ok ? stage[c].y : (part5 == 0 ? kFar : 0.0);
            lds[buf][ch] = v;
        }
    };
    if (ntiles > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    const int per = kLaneTile >> lw;  // records per lane per tile
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles)
            gload(t + 1);
        const int j0 = jbeg + t * kLaneTile;
        const double2 *L = lds[buf] + w * 5;
        const int step = W * 5;
        if (hi < j0 || lo >= j0 + kLaneTile) {
            double2 p0 = L[0], p1 = L[1], p2 = L[2], p3 = L[3], p4 = L[4];
            for (int k = 0; k < per; ++k) {
                const int nx = (k + 1 < per ? k + 1 : k) * step;
                const double2 n0 = L[nx + 0], n1 = L[nx + 1], n2 = L[nx + 2], n3 = L[nx + 3],
                              n4 = L[nx + 4];
                interact_f64<false>(b, p0, p1, p2, p3, p4, eps2, 0);
                p0 = n0; p1 = n1; p2 = n2; p3 = n3; p4 = n4;
            }
        } else {
            for (int k = 0; k < per; ++k) {
                const int e = k * step;
                interact_f64<true>(b, L[e + 0], L[e + 1], L[e + 2], L[e + 3], L[e + 4], eps2,
                                   j0 + w + k * W);
            }
        }
        if (t + 1 < ntiles)
            lstore(buf ^ 1);
        __syncthreads();
    }
}

// ------------------------------------------------------ pairwise (split) ----
// Same quantities with the paper's extended-precision idea applied the other way
// round: the coordinate difference is taken in float-float,
//   dx = (xh_j - xh_i) + (xl_j - xl_i)   (x = xh + xl, each FP32),
// so close pairs keep their relative accuracy; the rest of the algebra runs in FP32
// and the FP32 sums of every kFold bodies are added into FP64 accumulators.
struct I32 {
    float xh[3], xl[3], v[3], a[3];
    float t[10];    // FP32 sums of the current fold
    double acc[10]; // FP64 accumulators
    int self;
};

constexpr int kFold = 16;

template <bool MASK>
__device__ __forceinline__ void interact_f32(I32 &b, const float4 p0, const float4 p1,
                                             const float4 p2, const float4 p3, float eps2,
                                             int jglob)
{
    const float dx = (p0.x - b.xh[0]) + (p1.x - b.xl[0]);
    const float dy = (p0.y - b.xh[1]) + (p1.y - b.xl[1]);
    const float dz = (p0.z - b.xh[2]) + (p1.z - b.xl[2]);
    const float dvx = p2.x - b.v[0], dvy = p2.y - b.v[1], dvz = p2.z - b.v[2];
    const float dax = p3.x - b.a[0], day = p3.y - b.a[1], daz = p3.z - b.a[2];
    float mj = p0.w;
    float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
    if (MASK) {
        const bool self = (jglob == b.self);
        mj = self ? 0.0f : mj;
        r2 = self ? 1.0f : r2;
    }
    const float rv = __builtin_fmaf(dx, dvx, __builtin_fmaf(dy, dvy, dz * dvz));
    const float vvra = __builtin_fmaf(
        dvx, dvx,
        __builtin_fmaf(dvy, dvy,
                       __builtin_fmaf(dvz, dvz, __builtin_fmaf(dx, dax, __builtin_fmaf(dy, day, dz * daz)))));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float alpha = rv * rinv2;
    const float beta = __builtin_fmaf(alpha, alpha, vvra * rinv2);
    const float mr = mj * rinv;
    const float m3 = mr * rinv2;
    const float a3 = 3.0f * alpha;
    const float a6 = 6.0f * alpha;
    const float b3 = 3.0f * beta;
    b.t[0] = __builtin_fmaf(m3, dx, b.t[0]);
    b.t[1] = __builtin_fmaf(m3, dy, b.t[1]);
    b.t[2] = __builtin_fmaf(m3, dz, b.t[2]);
    const float wx = __builtin_fmaf(-a3, dx, dvx);
    const float wy = __builtin_fmaf(-a3, dy, dvy);
    const float wz = __builtin_fmaf(-a3, dz, dvz);
    b.t[3] = __builtin_fmaf(m3, wx, b.t[3]);
    b.t[4] = __builtin_fmaf(m3, wy, b.t[4]);
    b.t[5] = __builtin_fmaf(m3, wz, b.t[5]);
    const float ux = __builtin_fmaf(-a6, wx, __builtin_fmaf(-b3, dx, dax));
    const float uy = __builtin_fmaf(-a6, wy, __builtin_fmaf(-b3, dy, day));
    const float uz = __builtin_fmaf(-a6, wz, __builtin_fmaf(-b3, dz, daz));
    b.t[6] = __builtin_fmaf(m3, ux, b.t[6]);
    b.t[7] = __builtin_fmaf(m3, uy, b.t[7]);
    b.t[8] = __builtin_fmaf(m3, uz, b.t[8]);
    b.t[9] -= mr;
}

template <int IPL, int BS>
__device__ __forceinline__ void load_i_split(const float *__restrict__ jrec,
                                             const int32_t *__restrict__ act, int n_act, int ibase,
                                             int idx_lo, int idx_hi, I32 (&b)[IPL], int &lo,
                                             int &hi, bool &bad)
{
    lo = 0x7fffffff;
    hi = -1;
    bad = false;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + (int)threadIdx.x;
        int i = act[slot < n_act ? slot : n_act - 1];
        if (i < idx_lo || i >= idx_hi) {
            bad = true;
            i = idx_lo;
        }
        b[q].self = i;
        const float4 *r = reinterpret_cast<const float4 *>(jrec + (size_t)i * kRecF);
        const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
        b[q].xh[0] = r0.x; b[q].xh[1] = r0.y; b[q].xh[2] = r0.z;
        b[q].xl[0] = r1.x; b[q].xl[1] = r1.y; b[q].xl[2] = r1.z;
        b[q].v[0] = r2.x; b[q].v[1] = r2.y; b[q].v[2] = r2.z;
        b[q].a[0] = r3.x; b[q].a[1] = r3.y; b[q].a[2] = r3.z;
#pragma unroll
        for (int c = 0; c < 10; ++c) {
            b[q].acc[c] = 0.0;
            b[q].t[c] = 0.0f;
        }
        lo = min(lo, i);
        hi = max(hi, i);
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
}

template <int IPL, int NW, int TILE>
__device__ __forceinline__ void tiles_split(const float *__restrict__ jrec, int jbeg, int jend,
                                            I32 (&b)[IPL], int lo, int hi, float eps2,
                                            float4 (*lds)[TILE * 4])
{
    constexpr int BS = 64 * NW;
    constexpr int CH = TILE * 4;  // 16-byte chunks per tile
    static_assert(CH % BS == 0, "tile chunks must split evenly over the workgroup");
    static_assert(TILE % kFold == 0, "tile must be a multiple of the fold length");
    constexpr int CPT = CH / BS;
    const int tid = threadIdx.x;
    const float4 *__restrict__ src = reinterpret_cast<const float4 *>(jrec);
    const int ntiles = (jend - jbeg + TILE - 1) / TILE;
    float4 stage[CPT];
    int valid = 0;
    auto gload = [&](int t) {
        const int j0 = jbeg + t * TILE;
        valid = (jend - j0) * 4;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = c * BS + tid;
            stage[c] = src[ch < valid ? (size_t)j0 * 4 + ch : 0];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int ch = c * BS + tid;
            const bool ok = ch < valid;
            const bool first = (ch % 4) == 0;  // padding record {far, far, far, m = 0, 0 ...}
            float4 v;
            v.x = ok ? stage[c].x : (first ? 1.0e18f : 0.0f);
            v.y = ok ? stage[c].y : (first ? 1.0e18f : 0.0f);
            v.z = ok ? stage[c].z : (first ? 1.0e18f : 0.0f);
            v.w = ok ? stage[c].w : 0.0f;
            lds[buf][ch] = v;
        }
    };
    auto fold = [&]() {
#pragma unroll
        for (int q = 0; q < IPL; ++q)
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                b[q].acc[c] += (double)b[q].t[c];
                b[q].t[c] = 0.0f;
            }
    };
    if (ntiles > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles)
            gload(t + 1);
        const int j0 = jbeg + t * TILE;
        const float4 *L = lds[buf];
        const bool masked = !(hi < j0 || lo >= j0 + TILE) && wave_has_self(b, j0, TILE);
        for (int jf = 0; jf < TILE; jf += kFold) {
            if (!masked) {
#pragma unroll 4
                for (int jj = jf; jj < jf + kFold; ++jj) {
                    const float4 p0 = L[jj * 4 + 0], p1 = L[jj * 4 + 1], p2 = L[jj * 4 + 2],
                                 p3 = L[jj * 4 + 3];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f32<false>(b[q], p0, p1, p2, p3, eps2, 0);
                }
            } else {
                for (int jj = jf; jj < jf + kFold; ++jj) {
                    const float4 p0 = L[jj * 4 + 0], p1 = L[jj * 4 + 1], p2 = L[jj * 4 + 2],
                                 p3 = L[jj * 4 + 3];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f32<true>(b[q], p0, p1, p2, p3, eps2, j0 + jj);
                }
            }
            fold();
        }
        if (t + 1 < ntiles)
            lstore(buf ^ 1);
        __syncthreads();
    }
}

// ------------------------------------------------------- per-body predictor ----
// Taylor prediction to the block time (Nitadori & Makino 2008), h = t - t_i:
//   xp = x + h v + h^2/2 a + h^3/6 j + h^4/24 s + h^5/120 c, and likewise vp, ap,
// evaluated in nested form. Writes the 80-byte j-record {xp, vp, ap, m} of body i
// and, when jrec32 is not null, the 64-byte FP32 record with x split as hi + lo.
// Vectors are [3][stride] structure-of-arrays.
__device__ __forceinline__ void predict_body(const double *X, const double *V, const double *Ac,
                                             const double *Jk, const double *S, const double *C,
                                             const double *M, size_t stride, size_t i, double h,
                                             double *jrec, float *jrec32)
{
    const double h2 = h * 0.5, h3 = h / 3.0, h4 = h * 0.25, h5 = h / 5.0;
    double xp[3], vp[3], ap[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = (size_t)k * stride + i;
        const double x = X[e], v = V[e], a = Ac[e], jk = Jk[e], s = S[e], c = C[e];
        xp[k] = x + h * (v + h2 * (a + h3 * (jk + h4 * (s + h5 * c))));
        vp[k] = v + h * (a + h2 * (jk + h3 * (s + h4 * c)));
        ap[k] = a + h * (jk + h2 * (s + h3 * c));
    }
    const double m = M[i];
    double2 *r = reinterpret_cast<double2 *>(jrec + i * kRecD);
    r[0] = make_double2(xp[0], xp[1]);
    r[1] = make_double2(xp[2], vp[0]);
    r[2] = make_double2(vp[1], vp[2]);
    r[3] = make_double2(ap[0], ap[1]);
    r[4] = make_double2(ap[2], m);
    if (jrec32) {
        float hi[3], lo[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            hi[k] = (float)xp[k];
            lo[k] = (float)(xp[k] - (double)hi[k]);
        }
        float4 *f = reinterpret_cast<float4 *>(jrec32 + i * kRecF);
        f[0] = make_float4(hi[0], hi[1], hi[2], (float)m);
        f[1] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        f[2] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], 0.0f);
        f[3] = make_float4((float)ap[0], (float)ap[1], (float)ap[2], 0.0f);
    }
}

// ------------------------------------------------------- per-body corrector ----
// Sixth-order Hermite corrector (Nitadori & Makino 2008) of body i over h, from
// its old a0, j0, s0 and the new evaluation e[(0..8) * estride] (a1, j1, s1):
//   v1 = v0 + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1)
//   x1 = x0 + h/2 (v0 + v1) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1)
// and the 3rd, 4th and 5th derivatives of a at the end of the step from the quintic
// through (a, j, s) at both ends:
//   a3 = [ 60 (a1-a0) - h ( 36 j1 +  24 j0) + h^2 ( 9 s1 -  3 s0)] / h^3
//   a4 = [360 (a1-a0) - h (192 j1 + 168 j0) + h^2 (36 s1 - 24 s0)] / h^4
//   a5 = [720 (a1-a0) - 360 h (j1 + j0)     + 60 h^2 (s1 - s0)]    / h^5
// a3 becomes the crackle of the next prediction; |a4| and |a5| feed the step
// criterion. Returns false if any result is not finite.
// The corrector from a body's old x, v, a, j, s (k-th component at index k) and the
// new a, j, s in e[c * estride] (c = 0..8): new x, v, a, j, s, c = a3 and |a4|, |a5|.
// Returns false if any result is not finite.
__device__ __forceinline__ bool correct_core(const double (&x0)[3], const double (&v0)[3],
                                             const double (&a0)[3], const double (&j0)[3],
                                             const double (&s0)[3], const double *e, size_t estride,
                                             double h, double (&x1)[3], double (&v1)[3],
                                             double (&a1)[3], double (&j1)[3], double (&s1)[3],
                                             double (&d3)[3], double &a4n, double &a5n)
{
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    double a4sq = 0.0, a5sq = 0.0;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a1[k] = e[(size_t)(0 + k) * estride];
        j1[k] = e[(size_t)(3 + k) * estride];
        s1[k] = e[(size_t)(6 + k) * estride];
        v1[k] = v0[k] + h / 2.0 * (a0[k] + a1[k]) - h2 / 10.0 * (j1[k] - j0[k]) +
                h3 / 120.0 * (s0[k] + s1[k]);
        x1[k] = x0[k] + h / 2.0 * (v0[k] + v1[k]) - h2 / 10.0 * (a1[k] - a0[k]) +
                h3 / 120.0 * (j0[k] + j1[k]);
        d3[k] = (60.0 * (a1[k] - a0[k]) - h * (36.0 * j1[k] + 24.0 * j0[k]) +
                 h2 * (9.0 * s1[k] - 3.0 * s0[k])) / h3;
        const double d4 = (360.0 * (a1[k] - a0[k]) - h * (192.0 * j1[k] + 168.0 * j0[k]) +
                           h2 * (36.0 * s1[k] - 24.0 * s0[k])) / h4;
        const double d5 = (720.0 * (a1[k] - a0[k]) - 360.0 * h * (j1[k] + j0[k]) +
                           60.0 * h2 * (s1[k] - s0[k])) / h5;
        a4sq += d4 * d4;
        a5sq += d5 * d5;
        finite = finite && isfinite(x1[k]) && isfinite(v1[k]) && isfinite(d3[k]) && isfinite(d4) &&
                 isfinite(d5);
    }
    a4n = sqrt(a4sq);
    a5n = sqrt(a5sq);
    return finite;
}

// A body's old state, for correct_core (component k of body i at k * stride + i).
struct BodyOld {
    double x[3], v[3], a[3], j[3], s[3];
};

__device__ __forceinline__ BodyOld load_body_old(const double *X, const double *V, const double *Ac,
                                                 const double *Jk, const double *S, size_t stride,
                                                 size_t i)
{
    BodyOld b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t o = (size_t)k * stride + i;
        b.x[k] = X[o];
        b.v[k] = V[o];
        b.a[k] = Ac[o];
        b.j[k] = Jk[o];
        b.s[k] = S[o];
    }
    return b;
}

// The corrector of body i in place, from its stored state (arrays [3][stride]).
__device__ __forceinline__ bool correct_body(double *X, double *V, double *Ac, double *Jk, double *S,
                                             double *C, double *a4n, double *a5n, size_t stride,
                                             size_t i, const double *e, size_t estride, double h)
{
    const BodyOld o = load_body_old(X, V, Ac, Jk, S, stride, i);
    double x1[3], v1[3], a1[3], j1[3], s1[3], d3[3], a4, a5;
    const bool finite = correct_core(o.x, o.v, o.a, o.j, o.s, e, estride, h, x1, v1, a1, j1, s1, d3,
                                     a4, a5);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t q = (size_t)k * stride + i;
        X[q] = x1[k];
        V[q] = v1[k];
        Ac[q] = a1[k];
        Jk[q] = j1[k];
        S[q] = s1[k];
        C[q] = d3[k];
    }
    a4n[i] = a4;
    a5n[i] = a5;
    return finite;
}

// ------------------------------------------------------ per-body step levels ----
// Regular step: generalised Aarseth criterion of order 6 (Nitadori & Makino 2008),
//   Delta = eta [ (sqrt(|a||s|) + |j|) / (sqrt(|a3||a5|) + |a4|) ]^(1/3),
// decided without a cube root: level k fits when dt_k^3 <= eta^3 * ratio.
// Initial step: Delta = eta_init min(|a|/|j|, sqrt(|a|/|s|)).
// Block rules: shrink to any fitting level; grow by one level only when the body's
// time t is a multiple of the doubled step and the doubled step fits; at start-up
// the step must also divide t. A body that fits no level up to L is clamped to L
// and *dtmin is set. Contraction is off and the operation order follows the
// definition, so the integer level follows from correctly rounded IEEE operations.
__device__ inline double norm3v_nc(double x, double y, double z)
{
#pragma clang fp contract(off)
    return sqrt(x * x + y * y + z * z);
}

__device__ inline double norm3_nc(const double *p, size_t stride, size_t i)
{
    return norm3v_nc(p[i], p[stride + i], p[2 * stride + i]);
}

// The level rules from the norms |a|, |j|, |s|, |a3| and |a4|, |a5| (the last three
// used by the regular step only).
__device__ inline int level_from_norms(double an, double jn, double sn, double cn, double a4n,
                                       double a5n, int64_t t, int kold, int init, double eta,
                                       double eta_init, int dt_max_log2, int L, bool *dtmin)
{
#pragma clang fp contract(off)
    int kc = -1;
    if (init) {
        const double ra = (jn > 0.0) ? an / jn : INFINITY;
        const double rs = (sn > 0.0) ? sqrt(an / sn) : INFINITY;
        double d0 = eta_init * (ra < rs ? ra : rs);
        if (isnan(d0))
            d0 = INFINITY;
        for (int k = 0; k <= L; ++k)
            if (ldexp(1.0, dt_max_log2 - k) <= d0) {
                kc = k;
                break;
            }
    } else {
        const double num = sqrt(an * sn) + jn;
        const double den = sqrt(cn * a5n) + a4n;
        double qv = INFINITY;
        if (den > 0.0)
            qv = (eta * eta * eta) * (num / den);
        if (isnan(qv) || !(den > 0.0) || isinf(den))
            qv = INFINITY;
        for (int k = 0; k <= L; ++k)
            if (ldexp(1.0, 3 * (dt_max_log2 - k)) <= qv) {
                kc = k;
                break;
            }
    }
    *dtmin = false;
    if (kc < 0) {
        kc = L;
        *dtmin = true;
    }
    int knew;
    if (init) {
        knew = kc;
        while (knew < L && (t % ((int64_t)1 << (L - knew))) != 0)
            ++knew;
    } else if (kc > kold) {
        knew = kc;
    } else if (kold >= 1 && kc <= kold - 1 && (t % ((int64_t)1 << (L - kold + 1))) == 0) {
        knew = kold - 1;
    } else {
        knew = kold;
    }
    return knew;
}

// The level of body i from its stored a, j, s, c, |a4|, |a5|.
__device__ inline int level_for_body(const double *Ac, const double *Jk, const double *S,
                                     const double *C, const double *a4n, const double *a5n,
                                     size_t stride, size_t i, int64_t t, int kold, int init,
                                     double eta, double eta_init, int dt_max_log2, int L,
                                     bool *dtmin)
{
    const double an = norm3_nc(Ac, stride, i), jn = norm3_nc(Jk, stride, i),
                 sn = norm3_nc(S, stride, i);
    const double cn = init ? 0.0 : norm3_nc(C, stride, i);
    return level_from_norms(an, jn, sn, cn, init ? 0.0 : a4n[i], init ? 0.0 : a5n[i], t, kold,
                            init, eta, eta_init, dt_max_log2, L, dtmin);
}

}  // namespace nb
