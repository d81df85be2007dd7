// nbody_crackle.hip -- the pairwise evaluation extended by one derivative, crackle
// (the third time derivative of the acceleration), in FP64 on gfx950.
//
// For an active body i and every j != i, with predicted positions, velocities,
// accelerations and jerks (r, v, a, jj relative; R = r.r + eps^2), the terms of the
// plain evaluation plus
//   C = m3 jj - 9 alpha S - 9 beta J - 3 gamma A,
//   gamma = (3 v.a + r.jj) / R + alpha (3 beta - 4 alpha^2),
// the time derivative of S along r' = v, v' = a, a' = jj (the 6th-order Hermite
// scheme's derivative chain, Nitadori & Makino 2008, continued one order: what an
// exact initial third derivative, or an 8th-order scheme, needs). In the fused form
// of the plain kernel, J = m3 w and S = m3 u, so C = m3 z with
//   z = jj - 3 gamma r - 9 beta w - 9 alpha u,
// and every accumulation is again one FMA.
//
// Layout: the 80-byte j-records of the plain path plus a 32-byte jerk record
// {jx, jy, jz, 0} per body, staged together through LDS as seven 16-byte chunks.
#include "nb_device.h"
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kCrkTile = 256;     // j-records per LDS tile
constexpr int kCrkWaves = 4;      // waves per workgroup
constexpr int kCrkIPL = 2;        // active bodies per lane
constexpr int kCrkBS = 64 * kCrkWaves;
constexpr int kCrkComp = 13;      // a(3) j(3) s(3) c(3) phi

// Predicted jerk of every body at `tick`: jp = j + h s + h^2/2 c (the predictor's
// series for the jerk, stopped at the same crackle term).
__global__ __launch_bounds__(256) void k_predict_jerk(Arrays A, int64_t n, int64_t tick, double ts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double h = (double)(tick - A.tick[i]) * ts;
    double jp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t e = (int64_t)k * n + i;
        jp[k] = A.j[e] + h * (A.s[e] + 0.5 * h * A.c[e]);
    }
    double2 *r = reinterpret_cast<double2 *>(A.jrecj + i * 4);
    r[0] = make_double2(jp[0], jp[1]);
    r[1] = make_double2(jp[2], 0.0);
}

struct ICrk {
    double x[3], v[3], a[3], j[3];
    double acc[kCrkComp];
    int self;
};

template <bool MASK>
__device__ __forceinline__ void interact_crackle(ICrk &b, const double2 p0, const double2 p1,
                                                 const double2 p2, const double2 p3, const double2 p4,
                                                 const double2 q0, const double2 q1, double eps2, int jglob)
{
    const double dx = p0.x - b.x[0], dy = p0.y - b.x[1], dz = p1.x - b.x[2];
    const double dvx = p1.y - b.v[0], dvy = p2.x - b.v[1], dvz = p2.y - b.v[2];
    const double dax = p3.x - b.a[0], day = p3.y - b.a[1], daz = p4.x - b.a[2];
    const double djx = q0.x - b.j[0], djy = q0.y - b.j[1], djz = q1.x - b.j[2];
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
    const double va = __builtin_fma(dvx, dax, __builtin_fma(dvy, day, dvz * daz));
    const double rj = __builtin_fma(dx, djx, __builtin_fma(dy, djy, dz * djz));
    const double rinv = rsqrt_f64(r2);
    const double rinv2 = rinv * rinv;
    const double alpha = rv * rinv2;
    const double beta = __builtin_fma(alpha, alpha, vvra * rinv2);
    const double mr = mj * rinv;
    const double m3 = mr * rinv2;
    // gamma = (3 v.a + r.j) / R + alpha (3 beta - 4 alpha^2)
    const double g1 = __builtin_fma(3.0, va, rj) * rinv2;
    const double gamma = __builtin_fma(alpha, __builtin_fma(-4.0 * alpha, alpha, 3.0 * beta), g1);
    const double a3 = 3.0 * alpha, a6 = 6.0 * alpha, a9 = 9.0 * alpha;
    const double b3 = 3.0 * beta, b9 = 9.0 * beta, g3 = 3.0 * gamma;
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
    const double zx = __builtin_fma(-a9, ux, __builtin_fma(-b9, wx, __builtin_fma(-g3, dx, djx)));
    const double zy = __builtin_fma(-a9, uy, __builtin_fma(-b9, wy, __builtin_fma(-g3, dy, djy)));
    const double zz = __builtin_fma(-a9, uz, __builtin_fma(-b9, wz, __builtin_fma(-g3, dz, djz)));
    b.acc[9] = __builtin_fma(m3, zx, b.acc[9]);
    b.acc[10] = __builtin_fma(m3, zy, b.acc[10]);
    b.acc[11] = __builtin_fma(m3, zz, b.acc[11]);
    b.acc[12] -= mr;
}

// Two active bodies per lane (slots q and q + 256 of the workgroup's 512); grid
// (ceil(n_act / 512), S); split s sweeps the j-range [s jch, min(n, (s+1) jch)) in
// LDS tiles, each record read once for both bodies, and writes its partial sums to
// part[(s * 13 + c) * n_act + q] (or straight to out when S = 1).
__global__ __launch_bounds__(kCrkBS) void k_eval_crackle(Arrays A, int n, const int32_t *__restrict__ idx,
                                                         int n_act, double eps2, int jch, double *__restrict__ dst)
{
    __shared__ double2 lds[kCrkTile * 7];
    const int tid = threadIdx.x;
    const int sp = blockIdx.y;
    ICrk b[kCrkIPL];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int u = 0; u < kCrkIPL; ++u) {
        const int q = blockIdx.x * kCrkBS * kCrkIPL + u * kCrkBS + tid;
        int i = idx[q < n_act ? q : n_act - 1];
        i = (i < 0 || i >= n) ? 0 : i;  // indices are checked on the host
        const double2 *r = reinterpret_cast<const double2 *>(A.jrec + (size_t)i * kRecD);
        const double2 *rj = reinterpret_cast<const double2 *>(A.jrecj + (size_t)i * 4);
        const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4], j0 = rj[0], j1 = rj[1];
        b[u].x[0] = r0.x; b[u].x[1] = r0.y; b[u].x[2] = r1.x;
        b[u].v[0] = r1.y; b[u].v[1] = r2.x; b[u].v[2] = r2.y;
        b[u].a[0] = r3.x; b[u].a[1] = r3.y; b[u].a[2] = r4.x;
        b[u].j[0] = j0.x; b[u].j[1] = j0.y; b[u].j[2] = j1.x;
#pragma unroll
        for (int c = 0; c < kCrkComp; ++c)
            b[u].acc[c] = 0.0;
        b[u].self = i;
        lo = min(lo, i);
        hi = max(hi, i);
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    const int jbeg = sp * jch;
    const int jend = min(n, jbeg + jch);
    const double2 *src = reinterpret_cast<const double2 *>(A.jrec);
    const double2 *srcj = reinterpret_cast<const double2 *>(A.jrecj);
    for (int j0 = jbeg; j0 < jend; j0 += kCrkTile) {
        const int cnt = min(kCrkTile, jend - j0);
        // stage: chunk c of record r at lds[r * 7 + c]; padding records are far and massless
        for (int e = tid; e < kCrkTile * 7; e += kCrkBS) {
            const int r = e / 7, c = e - r * 7;
            double2 v;
            if (r < cnt)
                v = c < 5 ? src[(size_t)(j0 + r) * 5 + c] : srcj[(size_t)(j0 + r) * 2 + (c - 5)];
            else
                v = make_double2(c <= 1 ? kFar : 0.0, c == 0 ? kFar : 0.0);
            lds[e] = v;
        }
        __syncthreads();
        if (hi < j0 || lo >= j0 + kCrkTile) {
            for (int r = 0; r < kCrkTile; ++r) {
                const double2 *L = lds + r * 7;
                const double2 p0 = L[0], p1 = L[1], p2 = L[2], p3 = L[3], p4 = L[4], p5 = L[5], p6 = L[6];
#pragma unroll
                for (int u = 0; u < kCrkIPL; ++u)
                    interact_crackle<false>(b[u], p0, p1, p2, p3, p4, p5, p6, eps2, 0);
            }
        } else {
            for (int r = 0; r < kCrkTile; ++r) {
                const double2 *L = lds + r * 7;
                const double2 p0 = L[0], p1 = L[1], p2 = L[2], p3 = L[3], p4 = L[4], p5 = L[5], p6 = L[6];
#pragma unroll
                for (int u = 0; u < kCrkIPL; ++u)
                    interact_crackle<true>(b[u], p0, p1, p2, p3, p4, p5, p6, eps2, j0 + r);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kCrkIPL; ++u) {
        const int q = blockIdx.x * kCrkBS * kCrkIPL + u * kCrkBS + tid;
        if (q < n_act)
#pragma unroll
            for (int c = 0; c < kCrkComp; ++c)
                dst[((size_t)sp * kCrkComp + c) * n_act + q] = b[u].acc[c];
    }
}

// out[e] = sum over s of part[s * count + e], s ascending.
__global__ __launch_bounds__(256) void k_reduce_crackle(const double *__restrict__ part, int S, int64_t count,
                                                        double *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count)
        return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        acc += part[(size_t)s * count + e];
    out[e] = acc;
}

__global__ __launch_bounds__(256) void k_store_crackle(Arrays A, int64_t n, const double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        A.c[(int64_t)k * n + i] = out[(int64_t)(9 + k) * n + i];
}

unsigned blocks(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace

hipError_t launch_eval_crackle(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act, double eps,
                               int64_t partial_slots, int64_t tick, int dt_min_log2, double *out,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_predict_jerk, dim3(blocks(n, 256)), dim3(256), 0, st, A, n, tick,
                       ldexp(1.0, dt_min_log2));
    if (n_act == 0)
        return hipGetLastError();
    // j-splits for about 4096 waves, within the partial buffer (10 doubles per slot)
    const int64_t iblocks = (n_act + kCrkBS * kCrkIPL - 1) / (kCrkBS * kCrkIPL);
    int64_t S = (4096 + 4 * iblocks - 1) / (4 * iblocks);
    const int64_t tiles = (n + kCrkTile - 1) / kCrkTile;
    S = S < tiles ? S : tiles;
    const int64_t cap = (10 * partial_slots) / (kCrkComp * n_act);
    S = S < cap ? S : cap;
    S = S < 1 ? 1 : S;
    int64_t jch = (n + S - 1) / S;
    jch = (jch + kCrkTile - 1) / kCrkTile * kCrkTile;
    S = (n + jch - 1) / jch;
    double *dst = S == 1 ? out : A.part;
    hipLaunchKernelGGL(k_eval_crackle, dim3((unsigned)iblocks, (unsigned)S), dim3(kCrkBS), 0, st, A, (int)n,
                       idx, (int)n_act, eps * eps, (int)jch, dst);
    if (S > 1)
        hipLaunchKernelGGL(k_reduce_crackle, dim3(blocks(kCrkComp * n_act, 256)), dim3(256), 0, st,
                           (const double *)A.part, (int)S, kCrkComp * n_act, out);
    return hipGetLastError();
}

hipError_t launch_store_crackle(const Arrays &A, int64_t n, const double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_store_crackle, dim3(blocks(n, 256)), dim3(256), 0, st, A, n, out);
    return hipGetLastError();
}

}  // namespace nb
