// nbody_sym.hip -- evaluation of every body against every body (the full active set
// of a block step where all bodies are due, and the start-up passes), with each
// pair computed once and added to both bodies.
//
// The pairwise terms of the 6th-order Hermite scheme (Nitadori & Makino 2008; the
// paper's section "Code implementation") are antisymmetric in the pair apart from the
// mass: with r = x_j - x_i, v, a the relative predicted velocity and acceleration and
// R = r.r + eps^2, the quantities alpha = r.v / R and beta = (v.v + r.a) / R + alpha^2
// are unchanged when i and j swap, while r, v, a, w = v - 3 alpha r and
// u = a - 3 beta r - 6 alpha w change sign. So with q = R^(-3/2):
//   body i gains m_j q (r, w, u) and phi_i -= m_j R^(-1/2),
//   body j gains -m_i q (r, w, u) and phi_j -= m_i R^(-1/2).
// The m-independent part (differences, R^(-1/2), alpha, beta, w, u) is shared, so a
// pair costs about 65 VALU instructions for its two interactions instead of about 108.
//
// Decomposition. Bodies form blocks of B = NW * 64 * kSymIPL (a workgroup holds one
// block in registers, kSymIPL per lane), each cut into P parts of H = B / P bodies
// (P from 1 to 12, more for smaller systems so that there are enough units). A unit
// is (row block I, part of a block): the first P units of row I are the parts of
// block I itself (taken one-sided: every i of the block against every j of the part,
// self pair masked), then the parts of the blocks J > I (taken symmetrically). Units
// are numbered row by row. Workgroup w takes unit w first and then claims the next
// unit from a counter (consecutive units of one row reuse the row's bodies in
// registers), so a workgroup that runs ahead of the other on its CU takes more units
// instead of leaving that one to finish alone at half occupancy. The last units (one
// per workgroup at most) are each cut into F pieces of H / F records, claimed like
// units, so that the workgroups' last claims end closer together. Symmetric units
// stream the j-range through LDS tiles of 64 records; at step k lane l pairs its
// bodies with record (l + k) mod 64 of the tile, so within a wave each record is
// updated by one lane at a time and its running sum moves through LDS (read, add,
// write back) from lane to lane; each wave has its own sums, added in wave order when
// the tile is done (two sets of sums, used by alternate tiles, so that the next
// tile's steps start while this tile's sums are being added and stored).
//
// Partial sums: the i-sums of claimed item v (a unit or a piece) go to slot v of the
// row buffer; the j-sums of unit (I, J, part p) go to slot (J (J - 1) / 2 + I) P + p
// of the column buffer (a piece fills its own records of the slot). A
// reduction pass adds, for each body, the row slots of its block (in item order,
// dealt round-robin to four running sums so that their loads overlap) and likewise
// its column slots (in row order), combines the eight sums in a fixed pattern, and
// writes the result in the order of the index list. The slots depend on the unit,
// not on the workgroup that took it, and every sum has a fixed order, so results are
// bitwise reproducible.
#include "nb_internal.h"
#include "nb_math.h"

namespace nb {
namespace {

constexpr int kSymIPL = 3;    // bodies per lane
constexpr int kSymTile = 64;  // records per j-tile (one per lane of a wave)

__device__ __forceinline__ void raise_err(Status *stt, int word) { stt->err[word] = 1; }

struct SymBody {
    double x[3], v[3], a[3];
    double m;
    double acc[10];
    int self;
};

struct SymUnit {
    int row, col, part;  // blocks I (row) and J (col), part of J
};

// First unit of row r: P units per block of the row, blocks r ... nb - 1.
__device__ __forceinline__ int64_t row_start(int r, int nb, int P)
{
    return (int64_t)P * ((int64_t)r * nb - (int64_t)r * (r - 1) / 2);
}

// First claimed item of unit u (u = units: the number of items).
__device__ __forceinline__ int64_t item_of(int64_t u, int64_t split0, int fine)
{
    return u <= split0 ? u : split0 + (u - split0) * fine;
}

// Unit u -> (row, col, part).
__device__ __forceinline__ SymUnit decode_unit(int64_t u, int nb, int P)
{
    int I = 0;
    while (row_start(I + 1, nb, P) <= u)
        ++I;
    const int k = (int)(u - row_start(I, nb, P));
    SymUnit s;
    s.row = I;
    s.col = I + k / P;
    s.part = k - (k / P) * P;
    return s;
}

// The m-independent part of a pair and its two accumulations. r points from the
// register body (i) to the record (j).
template <bool SYM, bool MASK>
__device__ __forceinline__ void pair_sym(SymBody &b, const double2 p0, const double2 p1,
                                         const double2 p2, const double2 p3, const double2 p4,
                                         double eps2, int jglob, double (&jac)[10])
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
    const double rinv3 = rinv * rinv2;
    const double a3 = 3.0 * alpha;
    const double a6 = 6.0 * alpha;
    const double b3 = 3.0 * beta;
    const double wx = __builtin_fma(-a3, dx, dvx);
    const double wy = __builtin_fma(-a3, dy, dvy);
    const double wz = __builtin_fma(-a3, dz, dvz);
    const double ux = __builtin_fma(-a6, wx, __builtin_fma(-b3, dx, dax));
    const double uy = __builtin_fma(-a6, wy, __builtin_fma(-b3, dy, day));
    const double uz = __builtin_fma(-a6, wz, __builtin_fma(-b3, dz, daz));
    const double qj = mj * rinv3;
    b.acc[0] = __builtin_fma(qj, dx, b.acc[0]);
    b.acc[1] = __builtin_fma(qj, dy, b.acc[1]);
    b.acc[2] = __builtin_fma(qj, dz, b.acc[2]);
    b.acc[3] = __builtin_fma(qj, wx, b.acc[3]);
    b.acc[4] = __builtin_fma(qj, wy, b.acc[4]);
    b.acc[5] = __builtin_fma(qj, wz, b.acc[5]);
    b.acc[6] = __builtin_fma(qj, ux, b.acc[6]);
    b.acc[7] = __builtin_fma(qj, uy, b.acc[7]);
    b.acc[8] = __builtin_fma(qj, uz, b.acc[8]);
    b.acc[9] = __builtin_fma(-mj, rinv, b.acc[9]);
    if (SYM) {
        const double qi = b.m * rinv3;
        jac[0] = __builtin_fma(-qi, dx, jac[0]);
        jac[1] = __builtin_fma(-qi, dy, jac[1]);
        jac[2] = __builtin_fma(-qi, dz, jac[2]);
        jac[3] = __builtin_fma(-qi, wx, jac[3]);
        jac[4] = __builtin_fma(-qi, wy, jac[4]);
        jac[5] = __builtin_fma(-qi, wz, jac[5]);
        jac[6] = __builtin_fma(-qi, ux, jac[6]);
        jac[7] = __builtin_fma(-qi, uy, jac[7]);
        jac[8] = __builtin_fma(-qi, uz, jac[8]);
        jac[9] = __builtin_fma(-b.m, rinv, jac[9]);
    }
}

// Bodies of row block I into registers: body I*B + q*BS + tid for q < kSymIPL; a
// body index at or past n becomes a zero-mass body far away (its own sums are not
// written, its terms for the records vanish).
template <int BS>
__device__ __forceinline__ void load_row(const double2 *__restrict__ src, int n, int64_t first,
                                         SymBody (&b)[kSymIPL])
{
#pragma unroll
    for (int q = 0; q < kSymIPL; ++q) {
        const int64_t i = first + q * BS + threadIdx.x;
        const bool ok = i < n;
        const double2 *r = src + (size_t)(ok ? i : 0) * 5;
        const double2 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
        b[q].x[0] = ok ? r0.x : kFar;
        b[q].x[1] = ok ? r0.y : kFar;
        b[q].x[2] = ok ? r1.x : kFar;
        b[q].v[0] = r1.y; b[q].v[1] = r2.x; b[q].v[2] = r2.y;
        b[q].a[0] = r3.x; b[q].a[1] = r3.y; b[q].a[2] = r4.x;
        b[q].m = ok ? r4.y : 0.0;
        b[q].self = (int)i;
#pragma unroll
        for (int c = 0; c < 10; ++c)
            b[q].acc[c] = 0.0;
    }
}

// The symmetric evaluation kernel: a persistent grid of G workgroups over the claimed
// items (U units, the last of them in pieces).
// LDS: two j-tiles of 64 records (double-buffered) and, per wave, the running j-sums
// of the 64 records of a tile (two sets, alternating by tile).
template <int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_eval_sym(Arrays A, int n, int nb, int P, int64_t split0,
                                                    int fine, int64_t items, int G, double eps2,
                                                    double *__restrict__ rowbuf,
                                                    double *__restrict__ colbuf,
                                                    unsigned *__restrict__ claim)
{
    constexpr int BS = 64 * NW;
    constexpr int B = BS * kSymIPL;
    const int H = B / P;                         // records per unit
    constexpr int CH = kSymTile * 5;             // 16-byte chunks per tile
    __shared__ double2 tile[2][CH];
    __shared__ double jsum[2][NW][10][kSymTile];  // component-major: a wave's 64 lanes touch
                                               // 64 consecutive doubles per component
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double2 *__restrict__ src = reinterpret_cast<const double2 *>(A.jrec);
    __shared__ int64_t s_next;
    SymBody b[kSymIPL];
    int row = -1;
    // A tile of 64 whole records is copied from global memory straight into LDS
    // (each wave moves 64 chunks of 16 bytes per instruction, no registers held
    // while the steps run); a tile that ends past the last body is staged through
    // registers with zero-mass far-away records as padding, before the steps.
    auto tile_async = [&](int j0, int buf) {
        const double2 *g = src + (size_t)j0 * 5;
        for (int c = wave * 64; c < CH; c += BS)
            __builtin_amdgcn_global_load_lds(g + c + lane,
                                             (__attribute__((address_space(3))) void *)&tile[buf][c],
                                             16, 0, 0);
    };
    auto tile_padded = [&](int j0, int buf) {
        const int valid = (min(n, j0 + kSymTile) - j0) * 5;
        for (int ch = tid; ch < CH; ch += BS) {
            const bool ok = ch < valid;
            const double2 v = src[(size_t)j0 * 5 + (ok ? ch : 0)];
            const int part5 = ch % 5;
            double2 w;
            w.x = ok ? v.x : (part5 <= 1 ? kFar : 0.0);
            w.y = ok ? v.y : (part5 == 0 ? kFar : 0.0);
            tile[buf][ch] = w;
        }
    };
    auto tile_load = [&](int j0, int buf) {
        if (j0 + kSymTile <= n)
            tile_async(j0, buf);
    };
    auto flush_unit = [&](int64_t slot) {
        double *dst = rowbuf + (size_t)slot * 10 * B;
#pragma unroll
        for (int q = 0; q < kSymIPL; ++q) {
            const int r = q * BS + tid;
            if ((int64_t)row * B + r < n)
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    dst[(size_t)c * B + r] = b[q].acc[c];
#pragma unroll
            for (int c = 0; c < 10; ++c)
                b[q].acc[c] = 0.0;
        }
    };
    for (int64_t v = blockIdx.x; v < items;) {
        // item v: unit u whole, or piece f of F of it
        int64_t u = v;
        int f = 0, F = 1;
        if (v >= split0) {
            F = fine;
            u = split0 + (v - split0) / F;
            f = (int)(v - split0 - (u - split0) * F);
        }
        const SymUnit su = decode_unit(u, nb, P);
        if (su.row != row) {
            row = su.row;
            load_row<BS>(src, n, (int64_t)row * B, b);
        }
        const int pbeg = su.col * B + su.part * H;  // the part's first record
        const int jbeg = pbeg + f * (H / F);
        const int jend = min(n, jbeg + H / F);
        // a part past the last body has no records: its slot holds zeros
        if (jbeg < jend) {
        const bool sym = su.col != su.row;
        const int ntiles = (jend - jbeg + kSymTile - 1) / kSymTile;
        __syncthreads();  // the previous unit is done with the tiles
        tile_load(jbeg, 0);
        if (jbeg + kSymTile > n)
            tile_padded(jbeg, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1;
            const int j0 = jbeg + t * kSymTile;
            if (t + 1 < ntiles)
                tile_load(j0 + kSymTile, buf ^ 1);  // the buffer the previous tile used
            const double2 *L = tile[buf];
            if (sym) {
                // step 0: record `lane` starts its sums in this lane's registers
                {
                    double jac[10];
#pragma unroll
                    for (int c = 0; c < 10; ++c)
                        jac[c] = 0.0;
                    const double2 *p = L + lane * 5;
                    const double2 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3], p4 = p[4];
#pragma unroll
                    for (int q = 0; q < kSymIPL; ++q)
                        pair_sym<true, false>(b[q], p0, p1, p2, p3, p4, eps2, 0, jac);
#pragma unroll
                    for (int c = 0; c < 10; ++c)
                        jsum[buf][wave][c][lane] = jac[c];
                }
                for (int k = 1; k < kSymTile; ++k) {
                    const int r = (lane + k) & (kSymTile - 1);
                    const double2 *p = L + r * 5;
                    const double2 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3], p4 = p[4];
                    double jac[10];
#pragma unroll
                    for (int c = 0; c < 10; ++c)
                        jac[c] = jsum[buf][wave][c][r];
#pragma unroll
                    for (int q = 0; q < kSymIPL; ++q)
                        pair_sym<true, false>(b[q], p0, p1, p2, p3, p4, eps2, 0, jac);
#pragma unroll
                    for (int c = 0; c < 10; ++c)
                        jsum[buf][wave][c][r] = jac[c];
                }
            } else {
                // the row's own block: one-sided, self pair masked
                double unused[10];
                for (int k = 0; k < kSymTile; ++k) {
                    const int r = (lane + k) & (kSymTile - 1);
                    const double2 *p = L + r * 5;
                    const double2 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3], p4 = p[4];
#pragma unroll
                    for (int q = 0; q < kSymIPL; ++q)
                        pair_sym<false, true>(b[q], p0, p1, p2, p3, p4, eps2, j0 + r, unused);
                }
            }
            if (t + 1 < ntiles && j0 + 2 * kSymTile > n)
                tile_padded(j0 + kSymTile, buf ^ 1);
            __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into the next tile
            __syncthreads();
            if (sym) {
                // the waves' sums of each record, added in wave order, to this unit's
                // column slot
                double *dst = colbuf +
                              (((size_t)su.col * (su.col - 1) / 2 + su.row) * P + su.part) * 10 * H;
                for (int e = tid; e < kSymTile * 10; e += BS) {
                    const int c = e / kSymTile, r = e - c * kSymTile;
                    double s = jsum[buf][0][c][r];
#pragma unroll
                    for (int v = 1; v < NW; ++v)
                        s += jsum[buf][v][c][r];
                    const int j = j0 + r;
                    if (j < jend)
                        dst[(size_t)c * H + (j - pbeg)] = s;
                }
            }
        }
        }
        flush_unit(v);
        __syncthreads();  // every thread has read s_next
        if (tid == 0)
            s_next = G + (int64_t)atomicAdd(claim, 1u);
        __syncthreads();
        v = s_next;
    }
}

// A running sum with Neumaier's compensation: s + c carries the sum of the added
// values with the rounding of each addition kept in c.
struct CompSum {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x)
    {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
};

// Per (index-list entry, component): the row slots of the body's block and its
// column slots, each in four interleaved compensated running sums (the pass is bound
// by its loads, so the compensation is free and the result carries no rounding of
// this pass beyond the last addition), combined in a fixed pattern.
template <int B>
__global__ __launch_bounds__(256) void k_sym_reduce(Arrays A, int n, const int32_t *__restrict__ idx,
                                                    int n_act, int P, int64_t split0, int fine,
                                                    const double *__restrict__ rowbuf,
                                                    const double *__restrict__ colbuf,
                                                    double *__restrict__ out, double *__restrict__ out2)
{
    const int H = B / P;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)10 * n_act)
        return;
    const int c = (int)(e / n_act);
    const int q = (int)(e - (int64_t)c * n_act);
    int i = idx[q];
    if ((unsigned)i >= (unsigned)n) {
        raise_err(A.status, kErrIndex);
        i = 0;
    }
    const int nb = (n + B - 1) / B;
    const int K = i / B, r = i - K * B, part = r / H;
    // four running sums over slots 0, 1, 2, 3 mod 4 (their loads overlap), added
    // in a fixed pattern
    const int64_t v0 = item_of(row_start(K, nb, P), split0, fine);
    const double *row = rowbuf + ((size_t)v0 * 10 + c) * B + r;
    const int nrow = (int)(item_of(row_start(K + 1, nb, P), split0, fine) - v0);
    const size_t rs = (size_t)10 * B;
    CompSum s0, s1, s2, s3;
    int k = 0;
    for (; k + 3 < nrow; k += 4) {
        const double x0 = row[k * rs], x1 = row[(k + 1) * rs], x2 = row[(k + 2) * rs],
                     x3 = row[(k + 3) * rs];
        s0.add(x0);
        s1.add(x1);
        s2.add(x2);
        s3.add(x3);
    }
    for (; k < nrow; ++k)
        s0.add(row[k * rs]);
    const double *col = colbuf + (size_t)K * (K - 1) / 2 * P * 10 * H + (size_t)part * 10 * H +
                        (size_t)c * H + (r - part * H);
    const size_t cs = (size_t)P * 10 * H;
    CompSum t0, t1, t2, t3;
    int I = 0;
    for (; I + 3 < K; I += 4) {
        const double x0 = col[I * cs], x1 = col[(I + 1) * cs], x2 = col[(I + 2) * cs],
                     x3 = col[(I + 3) * cs];
        t0.add(x0);
        t1.add(x1);
        t2.add(x2);
        t3.add(x3);
    }
    for (; I < K; ++I)
        t0.add(col[I * cs]);
    CompSum tot;
    const CompSum *parts[8] = {&s0, &s1, &s2, &s3, &t0, &t1, &t2, &t3};
    double comp = 0.0;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        tot.add(parts[p]->s);
        comp += parts[p]->c;
    }
    const double s = tot.s + (tot.c + comp);
    out[(size_t)c * n_act + q] = s;
    if (out2)
        out2[(size_t)c * n_act + q] = s;
}

}  // namespace

// Geometry of the symmetric evaluation of n bodies by G workgroups.
// Parts per block: the fewest (longest units, fewest row partials) that still give
// every workgroup about seven units to claim. The last units, as many as there are
// workgroups and at most a quarter of all, are cut into pieces of 128 records (64
// when H is not a multiple of 128), so that the end of the launch, where the last
// claims finish, is short against the whole.
SymPlan plan_sym(int64_t n, int G)
{
    SymPlan P{};
    P.B = kSymWaves * 64 * kSymIPL;
    P.nb = (int)((n + P.B - 1) / P.B);
    const int64_t pairs = (int64_t)P.nb * (P.nb + 1) / 2;  // blocks (I, J >= I)
    static const int kParts[] = {1, 2, 3, 4, 6, 12};       // B / P a multiple of 64
    P.parts = 12;
    for (int p : kParts)
        if (p * pairs >= 7 * (int64_t)G) {
            P.parts = p;
            break;
        }
    P.units = P.parts * pairs;
    const int H = P.B / P.parts;
    P.fine = (H % 128 == 0 && H >= 256) ? H / 128 : (H >= 128 ? H / 64 : 1);
    int64_t tail = P.fine > 1 ? P.units / 4 : 0;
    tail = tail < G ? tail : G;
    P.split0 = P.units - tail;
    P.items = P.split0 + tail * P.fine;
    P.G = (int)(G < P.items ? G : P.items);
    P.row_slots = P.items * 10 * P.B;
    P.col_slots = (int64_t)P.nb * (P.nb - 1) / 2 * 10 * P.B;
    return P;
}

hipError_t launch_eval_sym(const Arrays &A, const SymPlan &P, int64_t n, const int32_t *idx,
                           int64_t n_act, double eps, double *rowbuf, double *colbuf,
                           unsigned *claim, double *dst, double *dst2, hipStream_t st)
{
    constexpr int B = kSymWaves * 64 * kSymIPL;
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(claim), 0, 1, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_eval_sym<kSymWaves>, dim3(P.G), dim3(64 * kSymWaves), 0, st, A, (int)n,
                       P.nb, P.parts, P.split0, P.fine, P.items, P.G, eps * eps, rowbuf, colbuf, claim);
    const int64_t count = 10 * n_act;
    hipLaunchKernelGGL(k_sym_reduce<B>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       A, (int)n, idx, (int)n_act, P.parts, P.split0, P.fine, rowbuf, colbuf, dst, dst2);
    return hipGetLastError();
}

}  // namespace nb
