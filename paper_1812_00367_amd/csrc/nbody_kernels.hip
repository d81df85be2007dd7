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

#include <math.h>

namespace nb {
namespace {

constexpr double kFar = 1.0e18;  // position of the zero-mass records that pad a tile

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

// 1/sqrt(x) to about one ulp: the hardware estimate v_rsq_f64 (relative error
// below 2^-24 measured on gfx950) followed by one third-order correction
// y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2, whose truncation error (5/16) e^3 is
// far below the FP64 rounding. (An FP32 estimate is as accurate and measured no
// faster once the conversions are counted.)
__device__ __forceinline__ double rsqrt_f64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x, y * y, 1.0);
    const double p = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y, e * p, y);
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

// ---------------------------------------------------------------- predictor ----
// Taylor prediction to the block time (Nitadori & Makino 2008), h = t - t_i:
//   xp = x + h v + h^2/2 a + h^3/6 j + h^4/24 s + h^5/120 c, and likewise vp, ap,
// evaluated in nested form. Writes the 80-byte j-record {xp, vp, ap, m} and, for the
// split path, the 64-byte FP32 record with x split as hi + lo.
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
    const double h2 = h * 0.5, h3 = h / 3.0, h4 = h * 0.25, h5 = h / 5.0;
    double xp[3], vp[3], ap[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = (size_t)k * n + i;
        const double x = A.x[e], v = A.v[e], a = A.a[e], jk = A.j[e], s = A.s[e], c = A.c[e];
        xp[k] = x + h * (v + h2 * (a + h3 * (jk + h4 * (s + h5 * c))));
        vp[k] = v + h * (a + h2 * (jk + h3 * (s + h4 * c)));
        ap[k] = a + h * (jk + h2 * (s + h3 * c));
    }
    const double m = A.m[i];
    double2 *r = reinterpret_cast<double2 *>(A.jrec + (size_t)i * kRecD);
    r[0] = make_double2(xp[0], xp[1]);
    r[1] = make_double2(xp[2], vp[0]);
    r[2] = make_double2(vp[1], vp[2]);
    r[3] = make_double2(ap[0], ap[1]);
    r[4] = make_double2(ap[2], m);
    if (split) {
        float hi[3], lo[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            hi[k] = (float)xp[k];
            lo[k] = (float)(xp[k] - (double)hi[k]);
        }
        float4 *f = reinterpret_cast<float4 *>(A.jrec32 + (size_t)i * kRecF);
        f[0] = make_float4(hi[0], hi[1], hi[2], (float)m);
        f[1] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        f[2] = make_float4((float)vp[0], (float)vp[1], (float)vp[2], 0.0f);
        f[3] = make_float4((float)ap[0], (float)ap[1], (float)ap[2], 0.0f);
    }
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
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = (size_t)k * n + i;
        A.a[e] = A.evalbuf[(size_t)(0 + k) * n + i];
        A.j[e] = A.evalbuf[(size_t)(3 + k) * n + i];
        A.s[e] = A.evalbuf[(size_t)(6 + k) * n + i];
        A.c[e] = 0.0;
    }
    A.phi[i] = A.evalbuf[(size_t)9 * n + i];
    A.a4n[i] = 0.0;
    A.a5n[i] = 0.0;
}

// --------------------------------------------------------- pairwise (FP64) ----
// For an active body i and every j != i (predicted quantities; softening eps):
//   r = x_j - x_i, v = v_j - v_i, a = a_j - a_i, R = r.r + eps^2,
//   m3 = m_j R^(-3/2), alpha = r.v / R, beta = (v.v + r.a) / R + alpha^2,
//   A = m3 r, J = m3 v - 3 alpha A, S = m3 a - 6 alpha J - 3 beta A, phi -= m_j R^(-1/2).
// They are accumulated in the equivalent fused form J = m3 w with w = v - 3 alpha r and
// S = m3 u with u = a - 3 beta r - 6 alpha w, so every accumulation is one FMA.
//
// Work decomposition: a workgroup of W waves holds W*64*IPL active bodies in
// registers (IPL per lane) and sweeps one j-range of `jchunk` bodies (one of S
// splits) tile by tile through LDS, double-buffered with register staging. Each
// workgroup writes its ten partial sums per body to part[s][10][n_act]; a second
// kernel adds the S splits in a fixed order. The self pair is masked only on tiles
// that contain one of the wave's own indices.
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

template <int IPL, int NW, int TILE>
__global__ __launch_bounds__(64 * NW) void k_eval_f64(Arrays A, int n, const int32_t *__restrict__ idx,
                                                      int n_act, double eps2, int jchunk,
                                                      double *__restrict__ part, int nsplit)
{
    constexpr int BS = 64 * NW;
    constexpr int CH = TILE * 5;  // 16-byte chunks per tile
    static_assert(CH % BS == 0, "tile chunks must split evenly over the workgroup");
    constexpr int CPT = CH / BS;
    __shared__ double2 lds[2][CH];

    const int tid = threadIdx.x;
    int ib, split;
    eval_block_coords(nsplit, ib, split);
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int ibase = ib * (BS * IPL);
    const double *__restrict__ jrec = A.jrec;

    I64 b[IPL];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + tid;
        int i = idx[slot < n_act ? slot : n_act - 1];
        if ((unsigned)i >= (unsigned)n) {
            raise_err(A.status, kErrIndex);
            i = 0;
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

    // Tile staging: every thread issues its CPT 16-byte loads unconditionally (an
    // out-of-range chunk reloads chunk 0) so they stay in flight during the
    // previous tile's arithmetic; padding is substituted when storing to LDS.
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
            const int part5 = ch % 5;  // padding record {far, far, far, 0 ... 0, m = 0}
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
        if (hi < j0 || lo >= j0 + TILE) {
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

#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + tid;
        if (slot < n_act) {
#pragma unroll
            for (int c = 0; c < 10; ++c)
                part[((size_t)split * 10 + c) * n_act + slot] = b[q].acc[c];
        }
    }
}

// ------------------------------------------------------ pairwise (split) ----
// Same quantities with the paper's extended-precision idea applied the other way
// round: the coordinate difference is taken in float-float,
//   dx = (xh_j - xh_i) + (xl_j - xl_i)   (x = xh + xl, each FP32),
// so close pairs keep their relative accuracy; the rest of the algebra runs in FP32
// and each tile's FP32 sums are added into FP64 accumulators (FP64 accumulation).
struct I32 {
    float xh[3], xl[3], v[3], a[3];
    float t[10];    // FP32 sums of the current tile
    double acc[10]; // FP64 accumulators
    int self;
};

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

// FP32 sub-sums are folded into FP64 every kFold j-bodies.
constexpr int kFold = 16;

template <int IPL, int NW, int TILE>
__global__ __launch_bounds__(64 * NW) void k_eval_split(Arrays A, int n, const int32_t *__restrict__ idx,
                                                        int n_act, float eps2, int jchunk,
                                                        double *__restrict__ part, int nsplit)
{
    constexpr int BS = 64 * NW;
    constexpr int CH = TILE * 4;  // 16-byte chunks per tile
    static_assert(CH % BS == 0, "tile chunks must split evenly over the workgroup");
    static_assert(TILE % kFold == 0, "tile must be a multiple of the fold length");
    constexpr int CPT = CH / BS;
    __shared__ float4 lds[2][CH];

    const int tid = threadIdx.x;
    int ib, split;
    eval_block_coords(nsplit, ib, split);
    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int ibase = ib * (BS * IPL);
    const float *__restrict__ jrec = A.jrec32;

    I32 b[IPL];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + tid;
        int i = idx[slot < n_act ? slot : n_act - 1];
        if ((unsigned)i >= (unsigned)n) {
            raise_err(A.status, kErrIndex);
            i = 0;
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
        const bool masked = !(hi < j0 || lo >= j0 + TILE);
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

#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = ibase + q * BS + tid;
        if (slot < n_act) {
#pragma unroll
            for (int c = 0; c < 10; ++c)
                part[((size_t)split * 10 + c) * n_act + slot] = b[q].acc[c];
        }
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
// Sixth-order Hermite corrector (Nitadori & Makino 2008) over h = t_next - t_i:
//   v1 = v0 + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1)
//   x1 = x0 + h/2 (v0 + v1) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1)
// and the 3rd, 4th and 5th derivatives of a at t_next from the quintic through
// (a, j, s) at both ends:
//   a3 = [ 60 (a1-a0) - h ( 36 j1 +  24 j0) + h^2 ( 9 s1 -  3 s0)] / h^3
//   a4 = [360 (a1-a0) - h (192 j1 + 168 j0) + h^2 (36 s1 - 24 s0)] / h^4
//   a5 = [720 (a1-a0) - 360 h (j1 + j0)     + 60 h^2 (s1 - s0)]    / h^5
// a3 becomes the crackle of the next prediction; |a4|, |a5| feed the step criterion.
__global__ __launch_bounds__(256) void k_correct(Arrays A, int n, const int32_t *__restrict__ idx,
                                                 int n_act, int64_t tick, double tick_size)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_act)
        return;
    const int i = idx[q];
    if ((unsigned)i >= (unsigned)n) {
        raise_err(A.status, kErrIndex);
        return;
    }
    const int64_t ti = A.tick[i];
    if (ti >= tick) {
        raise_err(A.status, kErrLevel);
        return;
    }
    const double h = (double)(tick - ti) * tick_size;
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    double a4sq = 0.0, a5sq = 0.0;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const size_t e = (size_t)k * n + i;
        const double a0 = A.a[e], j0 = A.j[e], s0 = A.s[e], v0 = A.v[e], x0 = A.x[e];
        const double a1 = A.evalbuf[(size_t)(0 + k) * n_act + q];
        const double j1 = A.evalbuf[(size_t)(3 + k) * n_act + q];
        const double s1 = A.evalbuf[(size_t)(6 + k) * n_act + q];
        const double v1 = v0 + h / 2.0 * (a0 + a1) - h2 / 10.0 * (j1 - j0) + h3 / 120.0 * (s0 + s1);
        const double x1 = x0 + h / 2.0 * (v0 + v1) - h2 / 10.0 * (a1 - a0) + h3 / 120.0 * (j0 + j1);
        const double d3 = (60.0 * (a1 - a0) - h * (36.0 * j1 + 24.0 * j0) + h2 * (9.0 * s1 - 3.0 * s0)) / h3;
        const double d4 =
            (360.0 * (a1 - a0) - h * (192.0 * j1 + 168.0 * j0) + h2 * (36.0 * s1 - 24.0 * s0)) / h4;
        const double d5 = (720.0 * (a1 - a0) - 360.0 * h * (j1 + j0) + 60.0 * h2 * (s1 - s0)) / h5;
        A.x[e] = x1;
        A.v[e] = v1;
        A.a[e] = a1;
        A.j[e] = j1;
        A.s[e] = s1;
        A.c[e] = d3;
        a4sq += d4 * d4;
        a5sq += d5 * d5;
        finite = finite && isfinite(x1) && isfinite(v1) && isfinite(d3) && isfinite(d4) && isfinite(d5);
    }
    A.a4n[i] = sqrt(a4sq);
    A.a5n[i] = sqrt(a5sq);
    A.phi[i] = A.evalbuf[(size_t)9 * n_act + q];
    A.tick[i] = tick;
    if (!finite)
        raise_err(A.status, kErrNumeric);
}

// -------------------------------------------------------------- step levels ----
// Regular step: generalised Aarseth criterion of order 6 (Nitadori & Makino 2008),
//   Delta = eta [ (sqrt(|a||s|) + |j|) / (sqrt(|a3||a5|) + |a4|) ]^(1/3),
// decided without a cube root: level k fits when dt_k^3 <= eta^3 * ratio.
// Initial step: Delta = eta_init min(|a|/|j|, sqrt(|a|/|s|)).
// Block rules: shrink to any fitting level; grow by one level only when the body's
// time is a multiple of the doubled step and the doubled step fits; at start-up the
// step must also divide the body's time. Below dt_min is an error (level clamped).
// Contraction is off and the operation order matches the definition, so the integer
// level follows from correctly rounded IEEE operations only.
__device__ double norm3_nc(const double *p, int n, int i)
{
#pragma clang fp contract(off)
    const double x = p[i], y = p[(size_t)n + i], z = p[2 * (size_t)n + i];
    return sqrt(x * x + y * y + z * z);
}

__global__ __launch_bounds__(256) void k_timesteps(Arrays A, int n, const int32_t *__restrict__ idx,
                                                   int n_act, int init, double eta, double eta_init,
                                                   int dt_max_log2, int L)
{
#pragma clang fp contract(off)
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_act)
        return;
    const int i = idx[q];
    if ((unsigned)i >= (unsigned)n) {
        raise_err(A.status, kErrIndex);
        return;
    }
    const double an = norm3_nc(A.a, n, i), jn = norm3_nc(A.j, n, i), sn = norm3_nc(A.s, n, i);
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
        const double cn = norm3_nc(A.c, n, i);
        const double num = sqrt(an * sn) + jn;
        const double den = sqrt(cn * A.a5n[i]) + A.a4n[i];
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
    if (kc < 0) {
        kc = L;
        raise_err(A.status, kErrDtMin);
    }
    const int64_t t = A.tick[i];
    int knew;
    if (init) {
        knew = kc;
        while (knew < L && (t % ((int64_t)1 << (L - knew))) != 0)
            ++knew;
    } else {
        const int kold = A.level[i];
        if (kc > kold)
            knew = kc;
        else if (kold >= 1 && kc <= kold - 1 && (t % ((int64_t)1 << (L - kold + 1))) == 0)
            knew = kold - 1;
        else
            knew = kold;
    }
    A.level[i] = knew;
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
    if (false) e = hipErrorInvalidValue;
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
