// nbody_group.hip -- evaluation of a partial active set (a block step in which only
// some bodies are due): a, j, s and phi of the listed bodies from every body, one-sided
// (the pairwise terms of the 6th-order Hermite scheme, section "Code implementation";
// the fused form of interact_f64).
//
// Decomposition. The active list is cut into groups of G bodies. A workgroup of NW
// waves takes one group and one j-split (a contiguous range of the predicted
// records); every wave of the workgroup holds the same G bodies, so the workgroup's
// waves share its range instead of each needing a range of its own:
//   - lane l of a wave holds bodies q P + l / W (q < IPL) of the group, P = 64 / W,
//     so G = IPL P (W lanes per body for small groups, one lane per body with IPL = 1
//     or 2 for large ones);
//   - the range streams through LDS tiles of 256 records (copied from global memory
//     straight into LDS, double-buffered), and lane slot k = wave W + (l mod W) takes
//     records k, k + NW W, k + 2 NW W, ... of each tile; or, for the smallest groups,
//     the lane slots read their records from memory directly;
//   - a body's sums are combined over its W lanes by a fixed butterfly and then over
//     the NW waves in wave order (in LDS).
// With one split the sums are the result. With S splits each workgroup writes its
// group's sums to slot s of part[s][10][n_act]; the partial buffer holds S n_act
// entries instead of the NW-fold more a wave per split would need. Then either a
// separate pass adds the S slots, or, when the group is small enough, the last
// workgroup of the group to finish does: it adds the slots in split order (fixed,
// whichever workgroup comes last), so one launch evaluates the set.
//
// Ordering of that hand-over: each thread stores its slot entries with agent-scope
// atomic stores and waits for them to complete; after a workgroup barrier, thread 0
// increments the group's counter with an agent-scope release; the workgroup that
// reads S - 1 takes an agent-scope acquire fence before reading the slots, and puts
// the counter back to zero for the next launch.
#include "nb_internal.h"
#include "nb_device.h"

namespace nb {
namespace {

constexpr int kGT = kGroupTile;  // records per LDS tile
constexpr int kGCH = kGT * 5;     // 16-byte chunks per tile

__device__ __forceinline__ void raise_err(Status *stt, int word) { stt->err[word] = 1; }

// The last workgroup of a group adds its S partial slots. Elements e = (component c,
// body b) of the group's G bodies; T threads per element (a power of two fixed by G,
// S and the workgroup size), thread t adding the slots s = t, t + T, ... in four
// running sums (slot by slot in turn), then the T results combined by a fixed tree in
// LDS. red must hold BS doubles.
template <int BS>
__device__ void group_tail(const double *__restrict__ part, int S, int n_act, int first, int G,
                           unsigned *ctr, double *__restrict__ dst, double *__restrict__ dst2,
                           double *red)
{
    const int tid = threadIdx.x;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's slot stores have completed
    __syncthreads();
    int last = 0;
    if (tid == 0) {
        const unsigned t = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == (unsigned)(S - 1));
    }
    if (!__syncthreads_or(last))
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int cnt = min(G, n_act - first);  // bodies of the group in the list
    const int E = 10 * cnt;
    int T = 1;
    while (2 * T * E <= BS && 2 * T <= S && T < 64)
        T *= 2;
    const int per = BS / T;  // elements per pass
    const int t = tid % T, el = tid / T;
    for (int base = 0; base < E; base += per) {
        const int e = base + el;
        const bool live = e < E;
        const int c = live ? e / cnt : 0, bb = live ? e - c * cnt : 0;
        const double *src = part + (size_t)c * n_act + first + bb;
        const size_t ss = (size_t)10 * n_act;  // one split further
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (live) {
            int s = t;
            for (; s + 7 * T < S; s += 8 * T) {
                const double v0 = src[s * ss], v1 = src[(s + T) * ss], v2 = src[(s + 2 * T) * ss],
                             v3 = src[(s + 3 * T) * ss], v4 = src[(s + 4 * T) * ss],
                             v5 = src[(s + 5 * T) * ss], v6 = src[(s + 6 * T) * ss],
                             v7 = src[(s + 7 * T) * ss];
                a0 += v0; a1 += v1; a2 += v2; a3 += v3;
                a0 += v4; a1 += v5; a2 += v6; a3 += v7;
            }
            for (; s + 3 * T < S; s += 4 * T) {
                const double v0 = src[s * ss], v1 = src[(s + T) * ss], v2 = src[(s + 2 * T) * ss],
                             v3 = src[(s + 3 * T) * ss];
                a0 += v0; a1 += v1; a2 += v2; a3 += v3;
            }
            for (; s < S; s += T)
                a0 += src[s * ss];
        }
        double acc = (a0 + a1) + (a2 + a3);
        if (T > 1) {
            red[tid] = acc;
            __syncthreads();
            for (int o = T >> 1; o > 0; o >>= 1) {
                if (t < o)
                    red[tid] += red[tid + o];
                __syncthreads();
            }
            acc = red[tid];
            __syncthreads();
        }
        if (live && t == 0) {
            const size_t o = (size_t)c * n_act + first + bb;
            dst[o] = acc;
            if (dst2)
                dst2[o] = acc;
        }
    }
    if (tid == 0)
        __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The group kernel. IPL bodies per lane (IPL = 2 only with W = 1); DIRECT: records read
// from memory by each lane slot (IPL = 1), else LDS tiles (NW W <= 256).
template <int IPL, int NW, bool DIRECT>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(IPL == 1 && NW == 8 && !DIRECT ? 4 : 1)))
void k_eval_grp(Arrays A, int n, const int32_t *__restrict__ idx,
                                                      int n_act, double eps2, int lw, int jchunk,
                                                      int nsplit, double *__restrict__ part,
                                                      unsigned *__restrict__ ctr,
                                                      double *__restrict__ dst,
                                                      double *__restrict__ dst2)
{
    static_assert(!DIRECT || IPL == 1, "direct reads hold one body per lane");
    constexpr int BS = 64 * NW;
    __shared__ double2 tile[2][kGCH];  // also the cross-wave sums and the tail's tree
    int g, split;
    eval_block_coords(nsplit, g, split);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = 1 << lw, P = 64 >> lw, w = lane & (W - 1), p = lane >> lw;
    const int G = IPL * P, first = g * G;
    const double2 *__restrict__ src = reinterpret_cast<const double2 *>(A.jrec);

    const int jbeg = split * jchunk;
    const int jend = min(n, jbeg + jchunk);
    const int stride = NW * W, k0 = wave * W + w;
    const int ntiles = (jend - jbeg + kGT - 1) / kGT;
    const int rpt = kGT / stride;  // records per lane slot per tile
    // a whole tile: 64 chunks of 16 bytes per wave instruction, global -> LDS
    auto tile_async = [&](int j0, int buf) {
        const double2 *gsrc = src + (size_t)j0 * 5;
        for (int c = wave * 64; c < kGCH; c += BS)
            __builtin_amdgcn_global_load_lds(gsrc + c + lane,
                                             (__attribute__((address_space(3))) void *)&tile[buf][c],
                                             16, 0, 0);
    };
    // the last, partial tile of the records: through registers, zero-mass far-away
    // records as padding
    auto tile_padded = [&](int j0, int buf) {
        const int valid = (min(n, j0 + kGT) - j0) * 5;
        for (int ch = tid; ch < kGCH; ch += BS) {
            const bool ok = ch < valid;
            const double2 v = src[(size_t)j0 * 5 + (ok ? ch : 0)];
            const int part5 = ch % 5;
            double2 u;
            u.x = ok ? v.x : (part5 <= 1 ? kFar : 0.0);
            u.y = ok ? v.y : (part5 == 0 ? kFar : 0.0);
            tile[buf][ch] = u;
        }
    };
    // the first tile (or the first records of a direct sweep) is requested before the
    // active bodies' records, so that the two memory round trips overlap
    DirectHead head{};
    if (DIRECT)
        head = direct_head(src, jbeg, jend, stride, k0);
    else if (ntiles > 0) {
        if (jbeg + kGT <= n)
            tile_async(jbeg, 0);
        else
            tile_padded(jbeg, 0);
    }

    I64 b[IPL];
    int lo = 0x7fffffff, hi = -1;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int slot = first + q * P + p;
        int i = idx[slot < n_act ? slot : n_act - 1];
        if ((unsigned)i >= (unsigned)n) {
            bad = true;
            i = 0;
        }
        b[q].self = i;
        const double2 *r = src + (size_t)i * 5;
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
    if (bad)
        raise_err(A.status, kErrIndex);
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);

    if constexpr (DIRECT) {
        I64 &one = reinterpret_cast<I64 &>(b);
        sweep_direct_f64(src, jbeg, jend, stride, k0, one, lo, hi, eps2, head);
    } else {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1;
            const int j0 = jbeg + t * kGT;
            const bool more = t + 1 < ntiles;
            if (more && j0 + 2 * kGT <= n)
                tile_async(j0 + kGT, buf ^ 1);  // the buffer the previous tile used
            const double2 *L = tile[buf];
            if ((hi < j0 || lo >= j0 + kGT) || !wave_has_self(b, j0, kGT)) {
                // records alternate between two register sets, so the next record's LDS
                // reads are in flight during this record's arithmetic
                const double2 *pr = L + k0 * 5;
                const int step = stride * 5;
                double2 a0 = pr[0], a1 = pr[1], a2 = pr[2], a3 = pr[3], a4 = pr[4];
                int m = 0;
                for (; m + 2 < rpt; m += 2) {
                    const double2 *pb = pr + (m + 1) * step;
                    const double2 b0 = pb[0], b1 = pb[1], b2 = pb[2], b3 = pb[3], b4 = pb[4];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<false>(b[q], a0, a1, a2, a3, a4, eps2, 0);
                    const double2 *pa = pb + step;
                    a0 = pa[0]; a1 = pa[1]; a2 = pa[2]; a3 = pa[3]; a4 = pa[4];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<false>(b[q], b0, b1, b2, b3, b4, eps2, 0);
                }
                if (m + 1 < rpt) {
                    const double2 *pb = pr + (m + 1) * step;
                    const double2 b0 = pb[0], b1 = pb[1], b2 = pb[2], b3 = pb[3], b4 = pb[4];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<false>(b[q], a0, a1, a2, a3, a4, eps2, 0);
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<false>(b[q], b0, b1, b2, b3, b4, eps2, 0);
                } else {
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<false>(b[q], a0, a1, a2, a3, a4, eps2, 0);
                }
            } else {
                for (int m = 0; m < rpt; ++m) {
                    const int r = k0 + m * stride;
                    const double2 *pr = L + r * 5;
                    const double2 p0 = pr[0], p1 = pr[1], p2 = pr[2], p3 = pr[3], p4 = pr[4];
#pragma unroll
                    for (int q = 0; q < IPL; ++q)
                        interact_f64<true>(b[q], p0, p1, p2, p3, p4, eps2, j0 + r);
                }
            }
            if (more && j0 + 2 * kGT > n)
                tile_padded(j0 + kGT, buf ^ 1);
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into the next tile
            __syncthreads();
        }
    }

    // a body's W lane sums (butterfly), then the NW waves in wave order through LDS,
    // one body set q at a time (NW x P x 10 doubles: at most the 40 KB of the tiles)
#pragma unroll
    for (int q = 0; q < IPL; ++q)
#pragma unroll
        for (int c = 0; c < 10; ++c)
            b[q].acc[c] = lane_butterfly(b[q].acc[c], W);
    double *red = reinterpret_cast<double *>(&tile[0][0]);
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        __syncthreads();  // the tiles (or the previous set's sums) are no longer read
        if (w == 0)
#pragma unroll
            for (int c = 0; c < 10; ++c)
                red[(wave * 10 + c) * P + p] = b[q].acc[c];
        __syncthreads();
        for (int e = tid; e < 10 * P; e += BS) {
            const int c = e / P, pp = e - c * P;
            double s = red[c * P + pp];
#pragma unroll
            for (int v = 1; v < NW; ++v)
                s += red[(v * 10 + c) * P + pp];
            const int slot = first + q * P + pp;
            if (slot < n_act) {
                if (nsplit == 1) {
                    dst[(size_t)c * n_act + slot] = s;
                    if (dst2)
                        dst2[(size_t)c * n_act + slot] = s;
                } else {
                    __hip_atomic_store(part + ((size_t)split * 10 + c) * n_act + slot, s,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    if (nsplit > 1 && ctr) {
        __syncthreads();  // the cross-wave sums are read: red is free for the tail
        group_tail<BS>(part, nsplit, n_act, first, G, ctr + g, dst, dst2, red);
    }
}

template <int IPL, int NW, bool DIRECT>
void launch_grp(dim3 grid, const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                int64_t n_act, double eps, unsigned *ctr, double *dst, double *dst2, hipStream_t st)
{
    hipLaunchKernelGGL((k_eval_grp<IPL, NW, DIRECT>), grid, dim3(64 * NW), 0, st, A, (int)n, idx,
                       (int)n_act, eps * eps, P.lw, P.jchunk, P.splits, A.part, ctr, dst, dst2);
}

}  // namespace

bool group_shape_ok(int pmax, int waves, int tile)
{
    if (waves != 4 && waves != 8)
        return false;
    if (pmax == 128)
        return tile == kGroupTile;  // two bodies per lane, one lane each
    if (pmax < 1 || pmax > 64 || (pmax & (pmax - 1)))
        return false;
    if (tile == 0)
        return true;
    // LDS tiles: the lane slots (waves x lanes per body) must divide the tile
    return tile == kGroupTile && waves * (64 / pmax) <= kGroupTile;
}

hipError_t launch_eval_group(const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                             int64_t n_act, double eps, unsigned *ctr, double *dst, double *dst2,
                             hipStream_t st)
{
    const bool xcd = P.splits > 1 && (P.splits % 8) == 0;
    const dim3 grid = xcd ? dim3(P.iblocks * P.splits, 1) : dim3(P.iblocks, P.splits);
    const bool two = P.ipl == -128, direct = P.tile == 0;
    if (P.waves == 4) {
        if (direct) launch_grp<1, 4, true>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
        else if (two) launch_grp<2, 4, false>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
        else launch_grp<1, 4, false>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
    } else if (P.waves == 8) {
        if (direct) launch_grp<1, 8, true>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
        else if (two) launch_grp<2, 8, false>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
        else launch_grp<1, 8, false>(grid, A, P, n, idx, n_act, eps, ctr, dst, dst2, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nb
