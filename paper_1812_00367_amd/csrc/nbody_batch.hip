// nbody_batch.hip -- many independent N-body systems ("jobs") of uneven size in one
// workspace, advanced together: every batch step gives each job its own next block
// step (its own block time and active set, the block-step scheme of the paper's
// section "Code implementation"), with a fixed sequence of four launches for all jobs
// and no host work in between:
//
//   k_bact     one workgroup per job: next block time, active list (ascending);
//   k_bpredict_plan  every body of every stepping job to its job's block time, and in
//              one more workgroup the plan: each stepping job's work split and the
//              prefix sums that place its work items, partial sums and active bodies;
//   k_beval    persistent waves taking work items (job, i-tile, j-chunk) until none
//              is left, class after class (three item classes in FP64, two in split);
//   k_bfinish  4 to 16 lanes per active body (from the job's S): fixed-order sum of
//              its partials, corrector, new step level.
//
// Pool layout: job j owns the contiguous body range [off_j, off_j + n_j) of a pool of
// `capacity` bodies; vectors are [3][capacity] structure-of-arrays and the j-records
// are the 80-byte (and 64-byte split) records of the single-system path.
//
// A job's split into work items depends only on its own (N, n_act), and every sum is
// taken in a fixed order, so its results are bitwise the same alone and in any mix.
#include "nbody.h"
#include "nb_device.h"
#include "nb_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

namespace nb {
namespace {

enum JobErr : int { kJobOk = 0, kJobNumeric = 1, kJobDtMin = 2, kJobLevel = 3 };

constexpr int kItemTile = 64;  // active bodies per work item at most (one wave)

// Per-step header written by k_plan.
// Work items come in three classes, each taken by its own persistent launch (each
// needs fewer registers than one kernel holding every sweep):
//   kClassTile: i-tiles of 64 active bodies of a job with fewer than kWideMin, one per
//               lane (or W lanes per body for a tail of 9..63), LDS-staged j-tiles;
//   kClassWide: i-tiles of 128 active bodies of a job with at least kWideMin, two per
//               lane (half the LDS reads per interaction; FP64 only);
//   kClassDirect: the tail tile of at most 8 active bodies, whose lanes read their
//               own records from global memory.
enum ItemClass : int { kClassTile = 0, kClassWide = 1, kClassDirect = 2, kClasses = 3 };

struct StepHdr {
    int64_t nitems[kClasses]; // work items of this step per class
    int64_t nfinw;        // waves of the finishing pass (each within one job)
    int64_t pslots;       // partial-sum slots used (x 10 doubles)
    int64_t inter;        // interactions accumulated over counted steps
    int64_t steps;        // counted steps in which some job advanced
    int32_t nplan;        // stepping jobs (entries of the plan)
    int32_t overflow;     // the partial-sum buffer was too small (never by construction)
    uint32_t counter[kClasses]; // next work item of each class (persistent evaluation)
    uint32_t pad[3];
};

struct Pool {
    double *m, *x, *v, *a, *j, *s, *c, *a4n, *a5n, *phi;
    int64_t *tick;
    int32_t *level;
    int2 *pblk;         // prediction blocks of the listed jobs: {job, first body} per kPlanBS bodies
    double *jrec;
    float *jrec32;
    int32_t *act;       // job j's active list (pool indices) at off_j
    double *part;
    int64_t part_cap;   // partial-sum slots
    // job table (by job id); j_nact, j_tnext and j_err are adjacent (one copy)
    int64_t *j_off, *j_n, *j_tend;
    int64_t *j_nact, *j_tnext;
    int32_t *j_err;
    // the next block time without a scan: the smallest t + dt of the bodies not due
    // in the job's last step (unchanged by it) and of its due bodies after their
    // correction; j_mok = 1 when both are up to date
    int64_t *j_mrest, *j_mact;
    int32_t *j_mok;
    // level-ordered active sets: perm lists each job's bodies by ascending step level
    // (at off_j), cnt[64 j + l] counts job j's bodies at level l, j_lact is the lowest
    // level of its last active list and j_lvmode is 1 when the job is kept that way,
    // 0 when it is scanned instead, -1 before its first active-set pass
    int32_t *perm, *cnt, *j_lact, *j_lvmode;
    // plan (by position among the stepping jobs)
    int32_t *pl_job, *pl_na, *pl_S, *pl_tiles, *pl_jch;
    int32_t *pl_keep;   // 1: the job keeps its running minima (more than kKnownMinN bodies)
    int64_t *pl_item0[kClasses], *pl_pbase;
    int64_t *pl_fw0;    // first finishing wave of each stepping job
    int64_t *pl_off, *pl_n;  // the job's body range (one load less for its work items)
    StepHdr *hdr;
    double *en_bsum;
    Status *status;
};

// -------------------------------------------------------- active selection ----
// One workgroup per listed job: tick_next = min over its bodies of t + dt, then the
// bodies due at tick_next in ascending order into act[off ...]; n_act = 0 when
// tick_next is beyond the job's end time or the job has failed.
constexpr int kBS = 1024;
constexpr int kBW = kBS / 64;
constexpr int kUnroll = 8;  // bodies per thread per round of the active-set scans
// Jobs larger than one round of the minimum scan take their next block time from the
// previous step instead (smaller ones scan: the bookkeeping would cost more than the
// round it saves).
constexpr int64_t kKnownMinN = (int64_t)kUnroll * kBS;
// Jobs larger than this keep their bodies in level order (bact_levels below): the
// active-set pass then reads only the last active list, except when that list is
// longer than kRankMax and the whole order is rebuilt by one workgroup (measured at
// 26 us for 16384 bodies and 83 us for 65536, against 6-8 us for a short list and
// about 20 us for the scan of 65536 bodies).
constexpr int64_t kLevelMinN = 2 * kKnownMinN;

// Active set from the level counts. In the block scheme every body's time t is a
// multiple of its step dt = 2^(L - level) ticks and the job's time T satisfies
// t <= T < t + dt, so t = floor(T / dt) dt and all bodies of one level are next due
// together, at (floor(T / dt) + 1) dt: the next block time is the smallest of these
// over the occupied levels, and the due bodies are those of every level at or above
// the lowest due one. perm keeps the job's bodies in the canonical order (level, index)
// (so the active list, its tail, is the same whatever the job's history, and a job
// resumed from a checkpoint steps bitwise like the uninterrupted one). After a step
// only the bodies of the last active list (the tail) have new levels, each one whose
// step divides the block time, so all above the levels of the other bodies (whose
// steps do not divide it, or they would have been due): a tail of at most kRankMax
// bodies is re-sorted in LDS (each body's rank among the tail bodies of its new level
// with smaller index); a longer one, and a job's first
// pass, rebuild the whole order by a counting sort over its bodies in index order
// (each wave a contiguous segment). Every body touched must sit on its level's grid
// at the job's time; if one does not (a state loaded with unrelated times), the job
// falls back to the scans (returns false).
constexpr int kRankMax = kBS;
constexpr int kGB = 8;  // groups of 64 bodies whose levels a wave loads at once

struct LevelLds {
    int hist[64];           // bodies per level of the tail (or of the job)
    int pos[64];            // next position of each level
    int seg[kBW][64];       // full pass: per wave and level, counts then positions
    int64_t key[kRankMax + 16];      // tail pass: (level << 32) | index in the job
    int flag;
};

// The lanes of the wave whose v (a value in [-1, 63]) equals this lane's: one ballot
// per bit of v (the value -1 has all bits set, and no lane holds 63 with it in use).
__device__ __forceinline__ unsigned long long same_value_lanes(int v)
{
    unsigned long long m = ~0ull;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        const bool bit = (v >> b) & 1;
        const unsigned long long bl = __ballot(bit);
        m &= bit ? bl : ~bl;
    }
    return m;
}

__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v |= __shfl_xor(v, off, 64);
    return v;
}

// The job's scalars, read together at the start of the active-set pass.
struct JobScalars {
    int64_t off, n, tnext, tend, nact;
    int err, lvmode, lact;
};

__device__ bool bact_levels(const Pool &P, int job, const JobScalars &J, int L, LevelLds &S,
                            int64_t *red)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t off = J.off, n = J.n;
    int32_t *cnt = P.cnt + (size_t)job * 64;
    const bool full = J.lvmode < 0 || J.nact > kRankMax;
    const int64_t m = full ? n : J.nact;  // bodies re-sorted: the last active list, or all
    const int64_t s0 = n - m;             // their first position in perm
    const int l0 = full ? 0 : J.lact;
    // the tail's bodies and the old counts are requested before anything waits
    int id = 0, lv = -1;
    int64_t tk = 0;
    if (!full && tid < m) {
        id = P.act[off + tid];
        lv = P.level[id];
        tk = P.tick[id];
    }
    const int c_old = (!full && wave == 0) ? cnt[lane] : 0;
    int64_t tref = J.tnext;
    if (J.lvmode < 0) {
        // a job's first pass: its time is its latest body's (a state loaded from a
        // checkpoint carries the bodies' own times)
        int64_t t = tref;
        for (int64_t k = tid; k < n; k += kBS) {
            const int64_t x = P.tick[off + k];
            t = x > t ? x : t;
        }
        t = -wave_min_i64(-t);
        if (lane == 0)
            red[wave] = t;
        __syncthreads();
        for (int w = 0; w < kBW; ++w)
            tref = red[w] > tref ? red[w] : tref;
        __syncthreads();
    }
    auto on_grid = [&](int l, int64_t t) {
        if (l < 0 || l > L || tref < 0)
            return false;
        const int64_t dt = (int64_t)1 << (L - l);
        return t == tref / dt * dt;
    };
    if (tid < 64)
        S.hist[tid] = 0;
    for (int e = tid; e < kBW * 64; e += kBS)
        (&S.seg[0][0])[e] = 0;
    if (tid == 0)
        S.flag = 0;
    __syncthreads();
    if (full) {
        // wave w: bodies [w sg, (w + 1) sg) in groups of 64, kGB groups' levels loaded
        // at once (on the first pass the times are checked too). In a group, the lanes
        // of one level are found by six ballots (one per bit of the level); the lowest
        // of them adds the group's count to the wave's counter of that level in LDS
        const int64_t sg = ((n + kBW - 1) / kBW + 63) / 64 * 64;
        const int64_t b0 = wave * sg, b1 = min(n, b0 + sg);
        const bool check = J.lvmode < 0;
        const unsigned long long below = (1ull << lane) - 1ull;
        int bad = 0;
        for (int64_t g0 = b0; g0 < b1; g0 += 64 * kGB) {
            int l[kGB];
            int64_t t[kGB];
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
                const int64_t k = g0 + u * 64 + lane;
                l[u] = k < b1 ? P.level[off + k] : -1;
                t[u] = (check && k < b1) ? P.tick[off + k] : 0;
            }
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
                if (l[u] >= 0 && (l[u] > L || (check && !on_grid(l[u], t[u])))) {
                    bad = 1;
                    l[u] = -1;
                }
                const unsigned long long same = same_value_lanes(l[u]);
                if (l[u] >= 0 && (same & below) == 0ull)
                    atomicAdd(&S.seg[wave][l[u]], __popcll(same));
            }
        }
        if (wave_max_i32(bad) && lane == 0)
            S.flag = 1;
        __syncthreads();
        if (S.flag)
            return false;
        if (wave == 0) {
            // level totals, their exclusive prefix, then each wave's start per level
            int tot = 0;
            for (int w = 0; w < kBW; ++w)
                tot += S.seg[w][lane];
            S.hist[lane] = tot;
            int incl = tot;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o)
                    incl += u;
            }
            int at = incl - tot;
            for (int w = 0; w < kBW; ++w) {
                const int c = S.seg[w][lane];
                S.seg[w][lane] = at;
                at += c;
            }
        }
        __syncthreads();
        for (int64_t g0 = b0; g0 < b1; g0 += 64 * kGB) {
            int l[kGB];
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
                const int64_t k = g0 + u * 64 + lane;
                l[u] = k < b1 ? P.level[off + k] : -1;
            }
            // the lowest lane of each level takes the group's positions of that level
            // from the wave's counter (the kGB groups' requests in flight together);
            // the others read their base from it
            unsigned long long same[kGB];
            int base[kGB];
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
                same[u] = same_value_lanes(l[u]);
                base[u] = 0;
                if (l[u] >= 0 && (same[u] & below) == 0ull)
                    base[u] = atomicAdd(&S.seg[wave][l[u]], __popcll(same[u]));
            }
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
                const int b = __shfl(base[u], __builtin_ctzll(same[u]), 64);
                if (l[u] >= 0)
                    P.perm[off + b + __popcll(same[u] & below)] = (int32_t)(g0 + u * 64 + lane + off);
            }
        }
    } else {
        if (tid < m) {
            if (on_grid(lv, tk)) {
                atomicAdd(&S.hist[lv], 1);
            } else {
                atomicOr(&S.flag, 1);
                lv = -1;
            }
            S.key[tid] = ((int64_t)lv << 32) | (int64_t)(uint32_t)(id - (int32_t)off);
        } else if (tid < ((m + 15) & ~15)) {
            S.key[tid] = INT64_MAX;  // padding of the last group of 16
        }
    }
    __syncthreads();
    if (wave == 0) {
        // the counts: below l0 the bodies before the tail (none at l0 or above) plus
        // the re-sorted bodies' new levels; the next block time; the due levels
        const int h = S.hist[lane];
        const int c = lane > L ? 0 : (lane < l0 ? c_old : 0) + h;
        if (!full) {
            // the tail must stay behind every other body in level order
            const int top = wave_max_i32(lane < l0 && c_old > 0 ? lane : -1);
            const int low = wave_min_i32(h > 0 ? lane : 64);
            if (lane == 0 && low <= top)
                S.flag = 1;
            int incl = h;
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o)
                    incl += u;
            }
            S.pos[lane] = (int)s0 + incl - h;
        }
        int64_t nx = INT64_MAX;
        if (c > 0) {
            const int64_t dt = (int64_t)1 << (L - lane);
            nx = (tref / dt + 1) * dt;
        }
        const int64_t tn = wave_min_i64(nx);
        const int lmin = wave_min_i32(c > 0 && nx == tn ? lane : 64);
        const int na = wave_sum_i32(lane >= lmin ? c : 0);
        if (lane == 0) {
            red[0] = tn;
            red[1] = na;
            red[2] = lmin;
        }
        S.hist[lane] = c;  // the new counts, stored below once the pass is known good
    }
    __syncthreads();
    if (S.flag)
        return false;
    const int64_t tn = red[0];
    const int lmin = (int)red[2];
    const bool skip = tn > J.tend || J.err != kJobOk;
    const int64_t nact = skip ? 0 : red[1];
    const int64_t start = n - nact;
    if (tid < 64)
        cnt[tid] = S.hist[tid];
    // act[off + k - start] = perm[off + k] for k in [start, e), eight loads in flight
    auto copy_due = [&](int64_t e) {
        for (int64_t k0 = start + tid; k0 < e; k0 += 8 * kBS) {
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = k0 + u * kBS;
                v[u] = k < e ? P.perm[off + k] : 0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = k0 + u * kBS;
                if (k < e)
                    P.act[off + k - start] = v[u];
            }
        }
    };
    if (full) {
        copy_due(n);
    } else {
        // bodies before the tail that are due now keep their places in perm
        copy_due(s0);
        if (tid < m) {
            // the tail: rank among the tail bodies of the same level with smaller index,
            // i.e. the keys in [lv << 32, own key), 16 keys per round
            const int64_t lo = (int64_t)lv << 32;
            const int64_t mine = lo | (int64_t)(uint32_t)(id - (int32_t)off);
            int r = 0;
            for (int e = 0; e < (int)m; e += 16) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int64_t k = S.key[e + u];
                    r += (k >= lo && k < mine) ? 1 : 0;
                }
            }
            const int64_t at = S.pos[lv] + r;
            P.perm[off + at] = id;
            if (at >= start)
                P.act[off + at - start] = id;
        }
    }
    if (tid == 0) {
        P.j_tnext[job] = tn;
        P.j_nact[job] = nact;
        P.j_lact[job] = skip ? 64 : lmin;
        P.j_lvmode[job] = 1;
    }
    return true;
}

__global__ __launch_bounds__(kBS) void k_bact(Pool P, const int32_t *__restrict__ jobs, int L)
{
    __shared__ int64_t red[kBW];
    __shared__ int wcu[kUnroll][kBW];
    __shared__ int sbad[kBW];
    __shared__ LevelLds s_lev;
    const int job = jobs[blockIdx.x];
    JobScalars J;
    J.err = P.j_err[job];
    J.tnext = P.j_tnext[job];
    J.tend = P.j_tend[job];
    J.off = P.j_off[job];
    J.n = P.j_n[job];
    J.nact = P.j_nact[job];
    J.lvmode = P.j_lvmode[job];
    J.lact = P.j_lact[job];
    // a failed job, or one whose last block time reached its end (every body is then
    // past it), does not step again: no scan
    if (J.err != kJobOk || J.tnext >= J.tend) {
        if (threadIdx.x == 0)
            P.j_nact[job] = 0;
        return;
    }
    const int64_t off = J.off, n = J.n;
    if (J.lvmode != 0) {
        if (bact_levels(P, job, J, L, s_lev, red))
            return;
        // the job is scanned from now on (every thread has read j_lvmode)
        __syncthreads();
        if (threadIdx.x == 0)
            P.j_lvmode[job] = 0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t mn = INT64_MAX;
    int badlevel = 0;
    // after a step of this job, t_next = min(t + dt) over its bodies is known without a
    // scan: the bodies that were not due kept their t and dt, and the due ones were
    // reduced by the finishing pass (the first step after admission scans)
    const bool known = P.j_mok[job] != 0;
    // kUnroll bodies per thread per round, their loads issued together
    for (int64_t k0 = threadIdx.x; !known && k0 < n; k0 += kUnroll * kBS) {
        int lv[kUnroll];
        int64_t tk[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t k = k0 + u * kBS;
            lv[u] = k < n ? P.level[off + k] : 0;
            tk[u] = k < n ? P.tick[off + k] : INT64_MAX;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (k0 + u * kBS >= n)
                continue;
            if (lv[u] < 0 || lv[u] > L) {
                badlevel = 1;
                lv[u] = L;
            }
            const int64_t e = tk[u] + ((int64_t)1 << (L - lv[u]));
            mn = e < mn ? e : mn;
        }
    }
    mn = wave_min_i64(mn);
    badlevel = wave_max_i32(badlevel);
    if (lane == 0) {
        red[wave] = mn;
        sbad[wave] = badlevel;
    }
    __syncthreads();
    // every thread takes the same decision from the same shared values
    int64_t tn = red[0];
    int anybad = sbad[0];
    for (int w = 1; w < kBW; ++w) {
        tn = red[w] < tn ? red[w] : tn;
        anybad |= sbad[w];
    }
    if (known) {
        const int64_t r = P.j_mrest[job], a = P.j_mact[job];
        tn = r < a ? r : a;
    }
    const int err0 = P.j_err[job];  // not written by this kernel before its end
    const bool skip = tn > P.j_tend[job] || err0 != kJobOk || anybad;
    int64_t base = 0;
    int64_t rest = INT64_MAX;  // smallest t + dt of the bodies not due at tn
    if (!skip) {
        // super-rounds of kUnroll chunks of kBS bodies: loads issued together, one
        // barrier pair per super-round; chunk u of a super-round starts after the due
        // bodies of chunks 0 .. u-1, and within a chunk the order is the thread order
        for (int64_t r0 = 0; r0 < n; r0 += kUnroll * kBS) {
            bool due[kUnroll];
            unsigned long long mask[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t k = r0 + u * kBS + threadIdx.x;
                int lv = k < n ? P.level[off + k] : 0;
                const int64_t tk = k < n ? P.tick[off + k] : 0;
                lv = (lv < 0 || lv > L) ? L : lv;
                const int64_t e = tk + ((int64_t)1 << (L - lv));
                due[u] = k < n && e == tn;
                if (k < n && !due[u])
                    rest = e < rest ? e : rest;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                mask[u] = __ballot(due[u]);
                if (lane == 0)
                    wcu[u][wave] = __popcll(mask[u]);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                int before = 0, tot = 0;
                for (int w = 0; w < kBW; ++w) {
                    const int c = wcu[u][w];
                    before += w < wave ? c : 0;
                    tot += c;
                }
                if (due[u])
                    P.act[off + base + before + __popcll(mask[u] & ((1ull << lane) - 1ull))] =
                        (int32_t)(off + r0 + u * kBS + threadIdx.x);
                base += tot;
            }
            __syncthreads();
        }
    }
    const bool keep = !skip && n > kKnownMinN;  // the same in every thread
    if (keep) {
        rest = wave_min_i64(rest);
        __syncthreads();  // red[] is reused
        if (lane == 0)
            red[wave] = rest;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < kBW; ++w)
                rest = red[w] < rest ? red[w] : rest;
    }
    if (threadIdx.x == 0) {
        P.j_tnext[job] = tn;
        P.j_nact[job] = skip ? 0 : base;
        if (anybad)
            P.j_err[job] = kJobLevel;
        // for the next step: the bodies not due now keep their t + dt; the finishing
        // pass lowers j_mact to the due bodies' new t + dt
        P.j_mrest[job] = rest;
        P.j_mact[job] = INT64_MAX;
        P.j_mok[job] = keep ? 1 : 0;
    }
}

// ------------------------------------------------------------- work split ----
// Lanes per active body of an i-tile with `rem` active bodies left: one lane each
// when rem >= 64 (every lane reads the same j-record: an LDS broadcast), otherwise
// the P = next power of two >= rem bodies share the wave, W = 64 / P lanes each, and
// lane w of a body takes records w, w + W, ... so the wave stays full for the
// one-to-few active bodies typical of a cluster's block steps.
__host__ __device__ inline int item_lanes(int64_t rem)
{
    if (rem >= 64)
        return 1;
    int p = 1;
    while (p < rem)
        p <<= 1;
    return 64 / p;
}

// The batch constants of the work split.
struct SplitCfg {
    int lane_recs;   // j-records per lane of a work item
    int target;      // work items per job at most (from j-chunks)
    int mul_tile, mul_wide, mul_direct;  // chunk-length factors of the three classes
    int64_t wide_min;                     // active bodies from which a job is wide
};

// Split of one job's evaluation: tiles = ceil(n_act / 64) i-tiles (of 128 for a wide
// job, n_act >= wide_min), S j-chunks of jch bodies. S gives every lane about
// `lane_recs` records (lane_recs 16 / W when W > 16 lanes share a body, so that a job
// with one to three active bodies still spreads over several waves), times the
// factor of the job's class: a wide job, a job whose active bodies take fewer than 8
// lanes each (tile items), or one whose take 8 or more (direct items). Longer chunks
// amortise each item's set-up and leave fewer partial sums for the finishing pass;
// shorter ones make more items. No more chunks than make `target` work items for
// the job. Depends on (n, n_act) and the batch constants only.

struct JobSplit {
    int64_t tiles, S, jch;
    bool wide;
};

__host__ __device__ inline JobSplit job_split(int64_t n, int64_t na, const SplitCfg &cfg)
{
    const int lane_recs = cfg.lane_recs, target = cfg.target;
    const int64_t wide_min = cfg.wide_min;
    JobSplit r;
    r.wide = na >= wide_min;
    const int64_t tw = r.wide ? 2 * kItemTile : kItemTile;
    r.tiles = (na + tw - 1) / tw;
    const int64_t W = r.wide ? 1 : item_lanes(na < 64 ? na : 64);
    const int64_t per = (int64_t)lane_recs * (r.wide ? cfg.mul_wide : W < 8 ? cfg.mul_tile * W
                                                                     : cfg.mul_direct * (W < 16 ? W : 16));
    int64_t S = (n + per - 1) / per;
    const int64_t cap = (target + r.tiles - 1) / r.tiles;
    S = S < cap ? S : cap;
    S = S < 1 ? 1 : S;
    int64_t jch = (n + S - 1) / S;
    jch = (jch + 63) / 64 * 64;
    r.jch = jch;
    r.S = (n + jch - 1) / jch;
    return r;
}

// Lanes per active body of the finishing pass: a power of two from 4 to 16, the fewest
// that leave each lane at most eight of the body's S partial sums (one set of loads in
// flight), 16 above S = 128 (32 or 64 lanes measured no faster: the butterfly grows).
// A function of S alone, like the sum's order.
constexpr int kFinMax = 16;
__host__ __device__ inline int fin_lanes(int64_t S)
{
    int f = 4;
    while (f < kFinMax && 8 * (int64_t)f < S)
        f <<= 1;
    return f;
}

// W lanes per body at or above this read their records straight from global memory
// (the W lanes of a body read W consecutive records per round, one contiguous
// block): an LDS tile would give each lane too few records to hide the next tile's
// load.
constexpr int kDirectW = 8;

// Active bodies from which an FP64 job's tiles hold 128 bodies, two per lane.
constexpr int64_t kWideMin = 128;

// Whether the last i-tile of a job with na active bodies in `tiles` tiles is taken by
// the direct class.
__host__ __device__ inline bool tail_direct(int64_t na, int64_t tiles)
{
    return item_lanes(na - (tiles - 1) * kItemTile) >= kDirectW;
}

// Block-wide exclusive scans of NV 64-bit values at once (NW waves): v[k] is
// replaced by its exclusive prefix and tot[k] receives the block total. Each wave
// scans its lanes, wave 0 scans the NW wave totals into pre, and every thread adds
// its wave's prefix: three barriers in all.
template <int NV, int NW>
__device__ __forceinline__ void block_scan(int64_t (&v)[NV], int64_t (&tot)[NV], int64_t (*scr)[NV],
                                           int64_t (*pre)[NV])
{
    static_assert(NW <= 32, "wave totals are scanned by one wave");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t inc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k)
        inc[k] = v[k];
    for (int o = 1; o < 64; o <<= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int64_t u = __shfl_up(inc[k], o, 64);
            if (lane >= o)
                inc[k] += u;
        }
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            scr[wave][k] = inc[k];
    __syncthreads();
    if (wave == 0) {
        // lane w <= NW: sum of the totals of waves before w (lane NW: all of them)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            int64_t x = lane < NW ? scr[lane][k] : 0;
            for (int o = 1; o < 32; o <<= 1) {
                const int64_t u = __shfl_up(x, o, 64);
                if (lane >= o)
                    x += u;
            }
            const int64_t ex = __shfl_up(x, 1, 64);
            if (lane <= NW)
                pre[lane][k] = lane == 0 ? 0 : ex;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        v[k] = pre[wave][k] + inc[k] - v[k];
        tot[k] = pre[NW][k];
    }
    __syncthreads();
}

// The step's plan over the listed jobs, by one workgroup of kPlanBS threads.
constexpr int kPlanBS = 256;

__device__ __forceinline__ void plan_jobs(const Pool &P, const int32_t *__restrict__ jobs, int njobs,
                                          const SplitCfg cfg, int count)
{
    constexpr int NW = kPlanBS / 64;
    __shared__ int64_t scr[NW][7], pre[NW + 1][7];
    int64_t c_plan = 0, c_it[kClasses] = {0, 0, 0}, c_ps = 0, c_inter = 0, c_fw = 0;
    for (int base = 0; base < njobs; base += kPlanBS) {
        const int p = base + (int)threadIdx.x;
        int job = -1;
        int64_t na = 0, n = 0, off = 0;
        JobSplit sp{0, 0, 0, false};
        if (p < njobs) {
            job = jobs[p];
            na = P.j_nact[job];
            n = P.j_n[job];
            off = P.j_off[job];
            if (na > 0)
                sp = job_split(n, na, cfg);
        }
        const bool on = na > 0;
        // items per class: a wide job's tiles; else full tiles (and a tail of 9..63)
        // in the tile class and a tail of at most 8 in the direct class
        const int64_t tail_d = on && !sp.wide && tail_direct(na, sp.tiles) ? 1 : 0;
        const int64_t n_items[kClasses] = {sp.wide ? 0 : (sp.tiles - tail_d) * sp.S,
                                           sp.wide ? sp.tiles * sp.S : 0, tail_d * sp.S};
        // finishing waves: fin_lanes(S) lanes per active body, a wave within one job
        const int64_t fw = on ? (na * fin_lanes(sp.S) + 63) / 64 : 0;
        // exclusive prefixes and totals of: stepping jobs, items of each class,
        // partial-sum slots, interactions, finishing waves
        int64_t x[7] = {on ? 1 : 0, n_items[0], n_items[1], n_items[2], sp.S * na, na * n, fw}, t[7];
        block_scan<7, NW>(x, t, scr, pre);
        const int64_t x_plan = x[0], x_it[kClasses] = {x[1], x[2], x[3]}, x_ps = x[4], x_fw = x[6];
        const int64_t t_plan = t[0], t_it[kClasses] = {t[1], t[2], t[3]}, t_ps = t[4], t_int = t[5],
                      t_fw = t[6];
        if (on) {
            const int64_t q = c_plan + x_plan;
            P.pl_job[q] = job;
            P.pl_na[q] = (int32_t)na;
            P.pl_S[q] = (int32_t)sp.S;
            P.pl_tiles[q] = (int32_t)sp.tiles;
            P.pl_jch[q] = (int32_t)sp.jch;
            P.pl_keep[q] = (n > kKnownMinN && P.j_lvmode[job] == 0) ? 1 : 0;
            for (int k = 0; k < kClasses; ++k)
                P.pl_item0[k][q] = c_it[k] + x_it[k];
            P.pl_pbase[q] = 10 * (c_ps + x_ps);
            P.pl_fw0[q] = c_fw + x_fw;
            P.pl_off[q] = off;
            P.pl_n[q] = n;
        }
        c_plan += t_plan;
        for (int k = 0; k < kClasses; ++k)
            c_it[k] += t_it[k];
        c_ps += t_ps;
        c_inter += t_int;
        c_fw += t_fw;
    }
    if (threadIdx.x == 0) {
        StepHdr *H = P.hdr;
        const bool over = c_ps > P.part_cap;
        H->overflow = over ? 1 : H->overflow;
        H->nplan = over ? 0 : (int32_t)c_plan;
        for (int k = 0; k < kClasses; ++k) {
            H->nitems[k] = over ? 0 : c_it[k];
            H->counter[k] = 0u;
        }
        H->nfinw = over ? 0 : c_fw;
        H->pslots = c_ps;
        if (count && !over) {
            H->inter += c_inter;
            H->steps += c_plan > 0 ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(kPlanBS) void k_plan(Pool P, const int32_t *__restrict__ jobs, int njobs,
                                                  SplitCfg cfg, int count)
{
    plan_jobs(P, jobs, njobs, cfg, count);
}

// Largest k in [0, count) with prefix[k] <= e (prefix ascending, prefix[0] = 0).
template <typename T>
__device__ __forceinline__ int find_entry(const T *__restrict__ prefix, int count, int64_t e)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The plan's prefix array in LDS when it has at most kPlanCache entries (a search
// there costs a few LDS reads instead of a chain of dependent global loads).
constexpr int kPlanCache = 1024;

__device__ __forceinline__ const int64_t *cache_prefix(const int64_t *__restrict__ g, int count,
                                                       int64_t *lds)
{
    if (count > kPlanCache)
        return g;
    for (int k = threadIdx.x; k < count; k += blockDim.x)
        lds[k] = g[k];
    __syncthreads();
    return lds;
}

// --------------------------------------------------------------- prediction ----
// Workgroup 0 builds the step's plan (it needs only the active counts); the others
// predict every body of a job that steps (n_act > 0) to its job's block time, one
// workgroup per kPlanBS bodies of each listed job (a table the host builds when the
// job list changes, so a step touches only the jobs' bodies, not the whole pool).
__global__ __launch_bounds__(kPlanBS) void k_bpredict_plan(Pool P, int64_t cap, double tick_size, int split,
                                                           const int32_t *__restrict__ jobs, int njobs,
                                                           SplitCfg cfg)
{
    if (blockIdx.x == 0) {
        plan_jobs(P, jobs, njobs, cfg, 1);
        return;
    }
    const int2 blk = P.pblk[blockIdx.x - 1];
    const int job = blk.x;
    const int64_t k = (int64_t)blk.y + threadIdx.x;
    if (k >= P.j_n[job] || P.j_nact[job] == 0)
        return;
    const int64_t i = P.j_off[job] + k;
    const int64_t tn = P.j_tnext[job], ti = P.tick[i];
    if (ti > tn) {
        P.j_err[job] = kJobLevel;
        return;
    }
    predict_body(P.x, P.v, P.a, P.j, P.s, P.c, P.m, (size_t)cap, (size_t)i,
                 (double)(tn - ti) * tick_size, P.jrec, split ? P.jrec32 : nullptr);
}

// One job's bodies [off, off + n) to a given time (start-up and energy).
__global__ __launch_bounds__(256) void k_bpredict_range(Pool P, int64_t cap, int64_t off, int64_t n,
                                                        int64_t tick, double tick_size, int split)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = off + k;
    const int64_t ti = P.tick[i];
    predict_body(P.x, P.v, P.a, P.j, P.s, P.c, P.m, (size_t)cap, (size_t)i,
                 (double)((tick > ti ? tick : ti) - ti) * tick_size, P.jrec, split ? P.jrec32 : nullptr);
}

// --------------------------------------------------------------- evaluation ----
// A work item of a job: i-tile `tile` (active slots tile*64 ...), j-chunk `sp`
// (bodies off + sp*jch ... off + min(n, (sp+1) jch)). Items of one j-chunk are
// adjacent in the item order, so the waves that take them at about the same time
// share that chunk in L2.
struct Item {
    int job, na, ibase, sp, W, lw, w, slot;
    int64_t off, n, pbase;
    int jbeg, jend;
};

template <int CLS>
__device__ __forceinline__ Item decode_item(const Pool &P, const int64_t *item0, int nplan, int64_t item)
{
    Item it;
    const int q = find_entry(item0, nplan, item);
    const int64_t local = item - item0[q];
    const int tiles = P.pl_tiles[q];
    it.job = P.pl_job[q];
    it.na = P.pl_na[q];
    if constexpr (CLS == kClassDirect) {
        // the job's last tile, one item per j-chunk
        it.sp = (int)local;
        it.ibase = (tiles - 1) * kItemTile;
    } else if constexpr (CLS == kClassWide) {
        it.sp = (int)(local / tiles);
        it.ibase = (int)(local - (int64_t)it.sp * tiles) * 2 * kItemTile;
    } else {
        const int tiles_a = tiles - (tail_direct(it.na, tiles) ? 1 : 0);
        it.sp = (int)(local / tiles_a);
        it.ibase = (int)(local - (int64_t)it.sp * tiles_a) * kItemTile;
    }
    it.pbase = P.pl_pbase[q];
    it.off = P.pl_off[q];
    it.n = P.pl_n[q];
    const int64_t jch = P.pl_jch[q];
    it.jbeg = (int)(it.off + (int64_t)it.sp * jch);
    it.jend = (int)min(it.off + it.n, (int64_t)it.jbeg + jch);
    it.W = CLS == kClassWide ? 1 : item_lanes(it.na - it.ibase);
    it.lw = __builtin_ctz(it.W);
    it.w = (int)threadIdx.x & (it.W - 1);
    it.slot = it.ibase + ((int)threadIdx.x >> it.lw);
    return it;
}

constexpr int kStageF = kItemTile * 4 / 64;  // ... per split tile

// Sum the W lanes of each body in a fixed butterfly and store the item's partial
// sums at part[pbase + (sp * 10 + c) * na + slot].
template <typename B>
__device__ __forceinline__ void finish_item(const Pool &P, B &b, const Item &it, bool bad)
{
#pragma unroll
    for (int c = 0; c < 10; ++c)
        b.acc[c] = lane_butterfly(b.acc[c], it.W);
    if (it.w == 0 && it.slot < it.na)
#pragma unroll
        for (int c = 0; c < 10; ++c)
            P.part[it.pbase + ((int64_t)it.sp * 10 + c) * it.na + it.slot] = b.acc[c];
    if (bad)
        P.j_err[it.job] = kJobLevel;
}

// The active body of this lane; an index outside the job's range is replaced by the
// job's first body and reported through *bad.
__device__ __forceinline__ int item_body(const Pool &P, const Item &it, bool *bad)
{
    int i = P.act[it.off + (it.slot < it.na ? it.slot : it.na - 1)];
    *bad = i < it.off || i >= it.off + it.n;
    return *bad ? (int)it.off : i;
}

// Work items are taken persistently, the classes of a launch in a fixed order. The
// first round is static: wave b takes item b of the classes' items laid end to end
// (so no wave waits on an atomic to start, and none is held back); a class with more
// items than the waves left for it hands the rest out from its counter, to waves that
// have finished their static item or the earlier classes.
__device__ __forceinline__ int64_t claim_item(const Pool &P, int cls, int64_t base)
{
    unsigned int got = 0;
    if (threadIdx.x == 0)
        got = atomicAdd(&P.hdr->counter[cls], 1u);
    return base + (int64_t)__shfl(got, 0, 64);
}

// First item of this wave in a class whose items start at position `before` of the
// launch's static round (nstat of them are static); -1 when the wave has none there.
__device__ __forceinline__ int64_t first_item(const Pool &P, int cls, int64_t nitems, int64_t before,
                                              int64_t *nstat)
{
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t room = G > before ? G - before : 0;
    *nstat = nitems < room ? nitems : room;
    if (b >= before && b - before < *nstat)
        return b - before;
    return *nstat < nitems ? claim_item(P, cls, *nstat) : -1;
}

// The items of one class; `before` = the items of the classes ahead of it.
template <int CLS>
__device__ __forceinline__ void eval_items_f64(const Pool &P, double eps2, double2 (*lds)[kItemTile * 5],
                                               int64_t *s_item0, int64_t before)
{
    const int64_t nitems = P.hdr->nitems[CLS];
    const int nplan = P.hdr->nplan;
    int64_t base;
    int64_t item = first_item(P, CLS, nitems, before, &base);
    if (item < 0 || item >= nitems)  // the other waves drain every item
        return;
    __syncthreads();  // the previous class is done with s_item0
    const int64_t *item0 = cache_prefix(P.pl_item0[CLS], nplan, s_item0);
    const double2 *__restrict__ src = reinterpret_cast<const double2 *>(P.jrec);
    while (item < nitems) {
        const Item it = decode_item<CLS>(P, item0, nplan, item);
        if constexpr (CLS == kClassWide) {
            // two active bodies per lane (slots ibase + lane and ibase + 64 + lane)
            I64 bw[2];
            int lo, hi;
            bool bad;
            load_i_f64<2, 64>(P.jrec, P.act + it.off, it.na, it.ibase, (int)it.off, (int)(it.off + it.n), bw,
                              lo, hi, bad);
            tiles_f64<2, 1, kItemTile>(P.jrec, it.jbeg, it.jend, bw, lo, hi, eps2,
                                       reinterpret_cast<double2 (*)[kItemTile * 5]>(&lds[0][0]));
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int slot = it.ibase + q * 64 + (int)threadIdx.x;
                if (slot < it.na)
#pragma unroll
                    for (int c = 0; c < 10; ++c)
                        P.part[it.pbase + ((int64_t)it.sp * 10 + c) * it.na + slot] = bw[q].acc[c];
            }
            if (bad)
                P.j_err[it.job] = kJobLevel;
        } else {
            bool bad;
            const int i = item_body(P, it, &bad);
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
            if constexpr (CLS == kClassDirect)
                sweep_direct_f64(src, it.jbeg, it.jend, it.W, it.w, b, lo, hi, eps2);
            else
                sweep_lds_f64(src, it.jbeg, it.jend, it.W, it.lw, it.w, b, lo, hi, eps2,
                              reinterpret_cast<double2 (*)[kItemTile * 5]>(&lds[0][0]));
            finish_item(P, b, it, bad);
        }
        item = base < nitems ? claim_item(P, CLS, base) : nitems;
    }
}

// All FP64 items of a step in one launch, class after class, so a wave that runs out
// of one class moves on while others finish theirs: first the direct class (few
// items, bound by load latency, which then overlaps the arithmetic of the others),
// then the wide class (the longest items), then the tile class.
__global__ __launch_bounds__(64) void k_beval_f64(Pool P, double eps2)
{
    __shared__ double2 lds[2][kItemTile * 5];
    __shared__ int64_t s_item0[kPlanCache];
    const int64_t nd = P.hdr->nitems[kClassDirect], nw = P.hdr->nitems[kClassWide];
    eval_items_f64<kClassDirect>(P, eps2, lds, s_item0, 0);
    eval_items_f64<kClassWide>(P, eps2, lds, s_item0, nd);
    eval_items_f64<kClassTile>(P, eps2, lds, s_item0, nd + nw);
}

// ------------------------------------------------------ split-precision path ----
struct Rec32 {
    float4 p0, p1, p2, p3;
};

__device__ __forceinline__ Rec32 load_rec32(const float4 *__restrict__ src, int j)
{
    const float4 *r = src + (size_t)j * 4;
    return Rec32{r[0], r[1], r[2], r[3]};
}

__device__ __forceinline__ void fold32(I32 &b)
{
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        b.acc[q] += (double)b.t[q];
        b.t[q] = 0.0f;
    }
}

// FP32 sums of kFold records of a lane are added into the FP64 accumulators.
__device__ __forceinline__ void sweep_direct_split(const float4 *__restrict__ src, int jbeg, int jend,
                                                   int W, int w, I32 &b, int lo, int hi, float eps2)
{
    const I32(&one)[1] = reinterpret_cast<const I32(&)[1]>(b);
    const int rounds = (jend - jbeg + W - 1) / W;
    auto idx = [&](int k) { return jbeg + k * W + w; };
    auto at = [&](int k) { const int j = idx(k); return j < jend ? j : jbeg; };
    Rec32 c = load_rec32(src, at(0));
    Rec32 nx = load_rec32(src, at(rounds > 1 ? 1 : 0));
    for (int k = 0; k < rounds; ++k) {
        const Rec32 f = load_rec32(src, at(k + 2 < rounds ? k + 2 : k));
        const int r0 = jbeg + k * W;
        if (r0 + W <= jend && ((hi < r0 || lo >= r0 + W) || !wave_has_self(one, r0, W))) {
            interact_f32<false>(b, c.p0, c.p1, c.p2, c.p3, eps2, 0);
        } else {
            const int j = idx(k);
            interact_f32<true>(b, c.p0, c.p1, c.p2, c.p3, eps2, j < jend ? j : b.self);
        }
        if (((k + 1) & (kFold - 1)) == 0)
            fold32(b);
        c = nx;
        nx = f;
    }
    fold32(b);
}

__device__ __forceinline__ void sweep_lds_split(const float4 *__restrict__ src, int jbeg, int jend,
                                                int W, int lw, int w, I32 &b, int lo, int hi, float eps2,
                                                float4 (*lds)[kItemTile * 4])
{
    const I32(&one)[1] = reinterpret_cast<const I32(&)[1]>(b);
    const int lane = threadIdx.x;
    const int ntiles = (jend - jbeg + kItemTile - 1) / kItemTile;
    float4 stage[kStageF];
    int valid = 0;
    auto gload = [&](int t) {
        const int j0 = jbeg + t * kItemTile;
        valid = (jend - j0) * 4;
#pragma unroll
        for (int c = 0; c < kStageF; ++c) {
            const int ch = c * 64 + lane;
            stage[c] = src[ch < valid ? (size_t)j0 * 4 + ch : 0];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int c = 0; c < kStageF; ++c) {
            const int ch = c * 64 + lane;
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
    if (ntiles > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    const int per = kItemTile >> lw;
    const int fold_tiles = per >= kFold ? 1 : kFold / per;
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles)
            gload(t + 1);
        const int j0 = jbeg + t * kItemTile;
        const float4 *L = lds[buf] + w * 4;
        const int step = W * 4;
        const bool masked = !(hi < j0 || lo >= j0 + kItemTile) && wave_has_self(one, j0, kItemTile);
        for (int k = 0; k < per; ++k) {
            const int e = k * step;
            if (masked)
                interact_f32<true>(b, L[e + 0], L[e + 1], L[e + 2], L[e + 3], eps2, j0 + w + k * W);
            else
                interact_f32<false>(b, L[e + 0], L[e + 1], L[e + 2], L[e + 3], eps2, 0);
            if (per >= kFold && ((k + 1) & (kFold - 1)) == 0)
                fold32(b);
        }
        if (per < kFold && ((t + 1) % fold_tiles) == 0)
            fold32(b);
        if (t + 1 < ntiles)
            lstore(buf ^ 1);
        __syncthreads();
    }
    fold32(b);
}

template <int CLS>
__device__ __forceinline__ void eval_items_split(const Pool &P, float eps2, float4 (*lds)[kItemTile * 4],
                                                 int64_t *s_item0, int64_t before)
{
    static_assert(CLS != kClassWide, "the split path has no wide class");
    constexpr bool DIRECT = CLS == kClassDirect;
    constexpr int cls = CLS;
    const int64_t nitems = P.hdr->nitems[cls];
    const int nplan = P.hdr->nplan;
    int64_t base;
    int64_t item = first_item(P, cls, nitems, before, &base);
    if (item < 0 || item >= nitems)  // the other waves drain every item
        return;
    __syncthreads();  // the previous class is done with s_item0
    const int64_t *item0 = cache_prefix(P.pl_item0[cls], nplan, s_item0);
    const float4 *__restrict__ src = reinterpret_cast<const float4 *>(P.jrec32);
    while (item < nitems) {
        const Item it = decode_item<CLS>(P, item0, nplan, item);
        bool bad;
        const int i = item_body(P, it, &bad);
        I32 b;
        {
            const float4 *r = src + (size_t)i * 4;
            const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
            b.xh[0] = r0.x; b.xh[1] = r0.y; b.xh[2] = r0.z;
            b.xl[0] = r1.x; b.xl[1] = r1.y; b.xl[2] = r1.z;
            b.v[0] = r2.x; b.v[1] = r2.y; b.v[2] = r2.z;
            b.a[0] = r3.x; b.a[1] = r3.y; b.a[2] = r3.z;
#pragma unroll
            for (int c = 0; c < 10; ++c) {
                b.acc[c] = 0.0;
                b.t[c] = 0.0f;
            }
            b.self = i;
        }
        const int lo = wave_min_i32(i), hi = wave_max_i32(i);
        if constexpr (DIRECT)
            sweep_direct_split(src, it.jbeg, it.jend, it.W, it.w, b, lo, hi, eps2);
        else
            sweep_lds_split(src, it.jbeg, it.jend, it.W, it.lw, it.w, b, lo, hi, eps2,
                            reinterpret_cast<float4 (*)[kItemTile * 4]>(&lds[0][0]));
        finish_item(P, b, it, bad);
        item = base < nitems ? claim_item(P, cls, base) : nitems;
    }
}

// All split-precision items of a step in one launch (direct class, then tile class,
// in the same way as the FP64 launch).
__global__ __launch_bounds__(64) void k_beval_split(Pool P, float eps2)
{
    __shared__ float4 lds[2][kItemTile * 4];
    __shared__ int64_t s_item0[kPlanCache];
    eval_items_split<kClassDirect>(P, eps2, lds, s_item0, 0);
    eval_items_split<kClassTile>(P, eps2, lds, s_item0, P.hdr->nitems[kClassDirect]);
}

// ------------------------------------------------- per active body: finishing ----
// One thread per active body of the step: the fixed-order sum of its S partials, then
//   kStartA:  the accelerations into the body's j-record (first start-up pass);
//   kStartB:  a, j, s, phi stored, c = a4 = a5 = 0, initial level (second pass);
//   kStep:    Hermite corrector over the step, phi and time, new level.
enum FinishMode : int { kStartA = 0, kStartB = 1, kStep = 2 };

// F = fin_lanes(S) lanes share one active body, and each wave of the pass stays within
// one job: the job's finishing waves (from the plan's prefix) take B = 64 / F of its
// active bodies each, lane l * B + b summing chunks l, l + F, ... of body b in
// ascending order, so the B lanes of each group read B consecutive slots of one chunk
// row. The F lane sums are then added by a fixed butterfly (l ^ F/2, ..., l ^ 1), and
// the lanes with l = 0 apply the result. The order depends on S only.
__global__ __launch_bounds__(256) void k_bfinish(Pool P, int64_t cap, int mode, double tick_size,
                                                 double eta, double eta_init, int dt_max_log2, int L)
{
    __shared__ int64_t s_fw0[kPlanCache];
    const int64_t nfw = P.hdr->nfinw;
    const int nplan = P.hdr->nplan;
    constexpr int per_block = 256 / 64;
    if ((int64_t)blockIdx.x * per_block >= nfw)
        return;
    const int64_t *fw0 = cache_prefix(P.pl_fw0, nplan, s_fw0);
    const int lane = (int)threadIdx.x & 63;
    const int wave = (int)threadIdx.x >> 6;
    // a wave-uniform loop over the pass's waves (shuffles inside)
    for (int64_t gw = (int64_t)blockIdx.x * per_block + wave; gw < nfw; gw += (int64_t)gridDim.x * per_block) {
        const int q = find_entry(fw0, nplan, gw);
        const int job = P.pl_job[q];
        const int64_t na = P.pl_na[q], pbase = P.pl_pbase[q];
        const int S = P.pl_S[q];
        const int F = fin_lanes(S), B = 64 / F;
        const int l = lane / B;
        const int64_t want = (gw - fw0[q]) * B + lane % B;
        const bool live = want < na;
        const int64_t slot = live ? want : na - 1;
        const bool keep = P.pl_keep[q] != 0;
        // a step's corrector: the body's index, time, level and old state are requested
        // before the partial sums, so the two sets of round trips overlap
        const bool owner = live && l == 0;
        int64_t i_pre = 0, ti_pre = 0, tn_pre = 0;
        int kold_pre = 0;
        BodyOld old{};
        if (mode == kStep && owner) {
            i_pre = P.act[P.pl_off[q] + slot];
            old = load_body_old(P.x, P.v, P.a, P.j, P.s, (size_t)cap, (size_t)i_pre);
            ti_pre = P.tick[i_pre];
            kold_pre = P.level[i_pre];
            tn_pre = P.j_tnext[job];
        }
        double ev[10];
#pragma unroll
        for (int c = 0; c < 10; ++c)
            ev[c] = 0.0;
        // chunks l, l + F, ... in ascending order; eight (then four) of them are loaded
        // at once so their round trips overlap (the additions keep the one-by-one order)
        int sp = l;
        for (; sp + 7 * F < S; sp += 8 * F) {
            double t[8][10];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double *src = P.part + pbase + (int64_t)(sp + u * F) * 10 * na + slot;
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    t[u][c] = src[(int64_t)c * na];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    ev[c] += t[u][c];
        }
        for (; sp + 3 * F < S; sp += 4 * F) {
            double t[4][10];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double *src = P.part + pbase + (int64_t)(sp + u * F) * 10 * na + slot;
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    t[u][c] = src[(int64_t)c * na];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    ev[c] += t[u][c];
        }
        for (; sp < S; sp += F) {
            const double *src = P.part + pbase + (int64_t)sp * 10 * na + slot;
#pragma unroll
            for (int c = 0; c < 10; ++c)
                ev[c] += src[(int64_t)c * na];
        }
        for (int o = 32; o >= B; o >>= 1)
#pragma unroll
            for (int c = 0; c < 10; ++c)
                ev[c] += __shfl_xor(ev[c], o, 64);
        int64_t nxt = INT64_MAX;  // the body's new t + dt (a completed step only)
        do {
            if (!live || l != 0)
                break;
            const int64_t i = mode == kStep ? i_pre : (int64_t)P.act[P.pl_off[q] + slot];
            if (mode == kStartA) {
                for (int c = 0; c < 3; ++c) {
                    P.jrec[i * kRecD + 6 + c] = ev[c];
                    if (P.jrec32)
                        P.jrec32[i * kRecF + 12 + c] = (float)ev[c];
                }
                break;
            }
            int init = 0;
            if (mode == kStartB) {
                for (int c = 0; c < 3; ++c) {
                    P.a[c * cap + i] = ev[0 + c];
                    P.j[c * cap + i] = ev[3 + c];
                    P.s[c * cap + i] = ev[6 + c];
                    P.c[c * cap + i] = 0.0;
                }
                P.a4n[i] = 0.0;
                P.a5n[i] = 0.0;
                P.phi[i] = ev[9];
                init = 1;
                bool finite = true;
#pragma unroll
                for (int c = 0; c < 10; ++c)
                    finite = finite && isfinite(ev[c]);
                if (!finite)  // e.g. two bodies at one place without softening
                    P.j_err[job] = kJobNumeric;
            } else {
                // the corrector and the new level from the values in registers
                const int64_t tn = tn_pre, ti = ti_pre;
                if (ti >= tn) {
                    P.j_err[job] = kJobLevel;
                    break;
                }
                double x1[3], v1[3], a1[3], j1[3], s1[3], d3[3], a4, a5;
                const bool ok = correct_core(old.x, old.v, old.a, old.j, old.s, ev, 1,
                                             (double)(tn - ti) * tick_size, x1, v1, a1, j1, s1, d3, a4,
                                             a5);
                for (int c = 0; c < 3; ++c) {
                    const size_t o = (size_t)c * cap + i;
                    P.x[o] = x1[c];
                    P.v[o] = v1[c];
                    P.a[o] = a1[c];
                    P.j[o] = j1[c];
                    P.s[o] = s1[c];
                    P.c[o] = d3[c];
                }
                P.a4n[i] = a4;
                P.a5n[i] = a5;
                P.phi[i] = ev[9];
                P.tick[i] = tn;
                if (!ok)
                    P.j_err[job] = kJobNumeric;
                bool dtmin;
                const int lv = level_from_norms(norm3v_nc(a1[0], a1[1], a1[2]),
                                                norm3v_nc(j1[0], j1[1], j1[2]),
                                                norm3v_nc(s1[0], s1[1], s1[2]),
                                                norm3v_nc(d3[0], d3[1], d3[2]), a4, a5, tn, kold_pre,
                                                0, eta, eta_init, dt_max_log2, L, &dtmin);
                P.level[i] = lv;
                if (dtmin)
                    P.j_err[job] = kJobDtMin;
                if (keep)
                    nxt = tn + ((int64_t)1 << (L - lv));
                break;
            }
            bool dtmin;
            const int lv = level_for_body(P.a, P.j, P.s, P.c, P.a4n, P.a5n, (size_t)cap, (size_t)i,
                                          P.tick[i], P.level[i], init, eta, eta_init, dt_max_log2, L,
                                          &dtmin);
            P.level[i] = lv;
            if (dtmin)
                P.j_err[job] = kJobDtMin;
            if (mode == kStep && keep)
                nxt = P.tick[i] + ((int64_t)1 << (L - lv));
        } while (false);
        if (mode == kStep) {
            // the due bodies' new t + dt, reduced per job for the next active-set
            // pass: one wave minimum and one atomic (the wave is within one job)
            const int64_t m = wave_min_i64(nxt);
            if (lane == 0 && m != INT64_MAX)
                atomicMin(reinterpret_cast<unsigned long long *>(P.j_mact + job), (unsigned long long)m);
        }
    }
}

// ------------------------------------------------------------- job set-up ----
__global__ __launch_bounds__(256) void k_bjob_init(Pool P, int job, int64_t off, int64_t n,
                                                   int64_t tick0)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        P.j_off[job] = off;
        P.j_n[job] = n;
        P.j_nact[job] = n;
        P.j_tnext[job] = tick0;
        P.j_err[job] = kJobOk;
        P.j_mok[job] = 0;  // the first step scans
        // a job of more than two scan rounds keeps its bodies in level order (its first
        // active-set pass sorts them); a smaller one is scanned
        P.j_lvmode[job] = n > kLevelMinN ? -1 : 0;
        P.j_lact[job] = 0;
    }
    if (k < n)
        P.act[off + k] = (int32_t)(off + k);
}

// Load a job's state from caller arrays laid out [3][n] into the pool ([3][cap]).
__global__ __launch_bounds__(256) void k_bload(Pool P, int64_t cap, int64_t off, int64_t n,
                                               const double *m, const double *x, const double *v,
                                               const double *a, const double *jk, const double *s,
                                               const double *c, const double *a4n, const double *a5n,
                                               const int64_t *tick, const int32_t *level, int64_t tick0)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = off + k;
    P.m[i] = m[k];
    for (int d = 0; d < 3; ++d) {
        P.x[d * cap + i] = x[d * n + k];
        P.v[d * cap + i] = v[d * n + k];
        P.a[d * cap + i] = a ? a[d * n + k] : 0.0;
        P.j[d * cap + i] = jk ? jk[d * n + k] : 0.0;
        P.s[d * cap + i] = s ? s[d * n + k] : 0.0;
        P.c[d * cap + i] = c ? c[d * n + k] : 0.0;
    }
    P.a4n[i] = a4n ? a4n[k] : 0.0;
    P.a5n[i] = a5n ? a5n[k] : 0.0;
    P.phi[i] = 0.0;
    P.tick[i] = tick ? tick[k] : tick0;
    P.level[i] = level ? level[k] : 0;
}

// Copy a job's state out of the pool into caller arrays ([3][n]); NULL skipped.
__global__ __launch_bounds__(256) void k_bstore(Pool P, int64_t cap, int64_t off, int64_t n, double *m,
                                                double *x, double *v, double *a, double *jk, double *s,
                                                double *c, double *a4n, double *a5n, double *phi,
                                                int64_t *tick, int32_t *level)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = off + k;
    if (m) m[k] = P.m[i];
    for (int d = 0; d < 3; ++d) {
        if (x) x[d * n + k] = P.x[d * cap + i];
        if (v) v[d * n + k] = P.v[d * cap + i];
        if (a) a[d * n + k] = P.a[d * cap + i];
        if (jk) jk[d * n + k] = P.j[d * cap + i];
        if (s) s[d * n + k] = P.s[d * cap + i];
        if (c) c[d * n + k] = P.c[d * cap + i];
    }
    if (a4n) a4n[k] = P.a4n[i];
    if (a5n) a5n[k] = P.a5n[i];
    if (phi) phi[k] = P.phi[i];
    if (tick) tick[k] = P.tick[i];
    if (level) level[k] = P.level[i];
}

__global__ __launch_bounds__(64) void k_hdr_reset(Pool P)
{
    if (threadIdx.x == 0) {
        StepHdr *H = P.hdr;
        for (int k = 0; k < kClasses; ++k) {
            H->nitems[k] = 0;
            H->counter[k] = 0u;
        }
        H->nfinw = 0;
        H->pslots = 0;
        H->inter = 0;
        H->steps = 0;
        H->nplan = 0;
        H->overflow = 0;
    }
}

unsigned nblk(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace
}  // namespace nb

using nb::Pool;

struct nb_batch {
    nb_batch_params p;
    hipStream_t st;
    Pool P;
    int64_t cap, partial_slots;
    nb::SplitCfg split_cfg;
    int eval_grid, finish_grid;
    char msg[512];
    // host job table
    std::vector<int64_t> off, n, tend;
    std::vector<char> alive;
    std::vector<std::pair<int64_t, int64_t>> free_ranges;  // (offset, length), sorted
    // pinned host staging
    int64_t *h_scalar;
    char *h_jobblk;     // mirror of j_nact | j_tnext | j_err
    nb::StepHdr *h_hdr;
    int32_t *h_jobs;
    int32_t *d_jobs, *d_one;
    int2 *h_pblk;       // prediction blocks of the listed jobs (host copy)
    int64_t npblk;
    nb::Status *h_status;
    bool jobs_dirty;    // the job list changed since it was last uploaded
    int njobs;
    // captured batch steps for multi-step calls: [0] one step, [1] kGraphSteps steps
    hipGraph_t graph[2];
    hipGraphExec_t gexec[2];
    bool graph_valid, no_graph;
    int64_t *h_nact() { return reinterpret_cast<int64_t *>(h_jobblk); }
    int64_t *h_tnext() { return reinterpret_cast<int64_t *>(h_jobblk) + p.max_jobs; }
    int32_t *h_err() { return reinterpret_cast<int32_t *>(h_jobblk + 16 * (size_t)p.max_jobs); }
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kDefaultLaneRecs = 64;
constexpr int kDefaultTarget = 2048;

int b_lane_recs(const nb_batch_params *p) { return p->jchunk > 0 ? p->jchunk : kDefaultLaneRecs; }
int b_target(const nb_batch_params *p) { return p->items_per_job > 0 ? p->items_per_job : kDefaultTarget; }

// Default chunk-length factors of the tile, wide and direct classes (measured on the
// 512-cluster ensemble and the serving mix, against 1: wide 4 gave +4 %, then tile 2
// +3 %; direct 2 or 1/2 were slower).
constexpr int kDefaultMul[3] = {2, 4, 1};

nb::SplitCfg b_split_cfg(const nb_batch_params *p)
{
    nb::SplitCfg c;
    c.lane_recs = b_lane_recs(p);
    c.target = b_target(p);
    const int32_t m[3] = {p->chunk_tile, p->chunk_wide, p->chunk_direct};
    c.mul_tile = m[0] > 0 ? m[0] : kDefaultMul[0];
    c.mul_wide = m[1] > 0 ? m[1] : kDefaultMul[1];
    c.mul_direct = m[2] > 0 ? m[2] : kDefaultMul[2];
    // the wide class (two bodies per lane) is FP64 only
    c.wide_min = p->precision == NB_SPLIT ? INT64_MAX : nb::kWideMin;
    return c;
}

// Partial-sum slots that every step fits by construction: a job with t i-tiles of w
// (64 or 128) bodies uses S n_act slots with S <= max(1, ceil(target / t)), i.e. at
// most n_act + w (target + 1).
int64_t b_partial_bound(const nb_batch_params *p)
{
    return 2 * p->capacity + 128 * ((int64_t)b_target(p) + 1) * p->max_jobs;
}

int64_t b_partial_slots(const nb_batch_params *p)
{
    const int64_t need = b_partial_bound(p);
    return p->partial_slots > need ? p->partial_slots : need;
}

// device workspace layout; returns bytes (base may be null to measure)
// Entries of the prediction-block table: one per kPlanBS bodies of each job, at most
// capacity / kPlanBS + max_jobs.
int64_t b_pblk_max(const nb_batch_params *p) { return p->capacity / nb::kPlanBS + p->max_jobs + 1; }

size_t b_layout(const nb_batch_params *p, Pool *P, int32_t **d_jobs, int32_t **d_one, char *base)
{
    const size_t cap = (size_t)p->capacity, J = (size_t)p->max_jobs;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = al256(off);
        void *r = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return r;
    };
    const bool split = p->precision == NB_SPLIT;
    const int64_t ps = b_partial_slots(p);
    P->m = (double *)take(8 * cap);
    P->x = (double *)take(24 * cap);
    P->v = (double *)take(24 * cap);
    P->a = (double *)take(24 * cap);
    P->j = (double *)take(24 * cap);
    P->s = (double *)take(24 * cap);
    P->c = (double *)take(24 * cap);
    P->a4n = (double *)take(8 * cap);
    P->a5n = (double *)take(8 * cap);
    P->phi = (double *)take(8 * cap);
    P->tick = (int64_t *)take(8 * cap);
    P->level = (int32_t *)take(4 * cap);
    P->pblk = (int2 *)take(8 * (size_t)b_pblk_max(p));
    P->jrec = (double *)take(8 * nb::kRecD * cap);
    P->jrec32 = split ? (float *)take(4 * nb::kRecF * cap) : nullptr;
    P->act = (int32_t *)take(4 * cap);
    P->part = (double *)take(80 * (size_t)ps);
    P->part_cap = ps;
    P->j_off = (int64_t *)take(8 * J);
    P->j_n = (int64_t *)take(8 * J);
    P->j_tend = (int64_t *)take(8 * J);
    char *blk = (char *)take(20 * J);
    P->j_nact = (int64_t *)blk;
    P->j_tnext = blk ? (int64_t *)(blk + 8 * J) : nullptr;
    P->j_err = blk ? (int32_t *)(blk + 16 * J) : nullptr;
    P->j_mrest = (int64_t *)take(8 * J);
    P->j_mact = (int64_t *)take(8 * J);
    P->j_mok = (int32_t *)take(4 * J);
    P->perm = (int32_t *)take(4 * cap);
    P->cnt = (int32_t *)take(4 * 64 * J);
    P->j_lact = (int32_t *)take(4 * J);
    P->j_lvmode = (int32_t *)take(4 * J);
    P->pl_job = (int32_t *)take(4 * J);
    P->pl_na = (int32_t *)take(4 * J);
    P->pl_S = (int32_t *)take(4 * J);
    P->pl_tiles = (int32_t *)take(4 * J);
    P->pl_jch = (int32_t *)take(4 * J);
    for (int k = 0; k < nb::kClasses; ++k)
        P->pl_item0[k] = (int64_t *)take(8 * J);
    P->pl_keep = (int32_t *)take(4 * J);
    P->pl_pbase = (int64_t *)take(8 * J);
    P->pl_fw0 = (int64_t *)take(8 * J);
    P->pl_off = (int64_t *)take(8 * J);
    P->pl_n = (int64_t *)take(8 * J);
    P->hdr = (nb::StepHdr *)take(sizeof(nb::StepHdr));
    P->en_bsum = (double *)take(16 * (size_t)nb::en_blocks(p->capacity));
    P->status = (nb::Status *)take(sizeof(nb::Status));
    *d_jobs = (int32_t *)take(4 * J);
    *d_one = (int32_t *)take(4);
    return al256(off);
}

nb_status bfail(nb_batch *b, nb_status s, const char *fmt, ...)
{
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(b->msg, sizeof b->msg, fmt, ap);
        va_end(ap);
    }
    return s;
}

#define B_HIP(b, call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), NB_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

const char *b_check_params(const nb_batch_params *p)
{
    if (!p) return "params is NULL";
    if (p->capacity < 1 || p->capacity > ((int64_t)1 << 30)) return "capacity must be in [1, 2^30]";
    if (p->max_jobs < 1 || p->max_jobs > (1 << 16)) return "max_jobs must be in [1, 65536]";
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return "eps must be finite and >= 0";
    if (!(p->eta > 0.0) || !isfinite(p->eta) || !(p->eta_init > 0.0) || !isfinite(p->eta_init))
        return "eta and eta_init must be finite and > 0";
    if (p->dt_max_log2 > 100 || p->dt_min_log2 < -200) return "dt_max_log2 <= 100 and dt_min_log2 >= -200";
    const int L = p->dt_max_log2 - p->dt_min_log2;
    if (L < 0 || L > 62) return "need 0 <= dt_max_log2 - dt_min_log2 <= 62";
    if (p->precision != NB_FP64 && p->precision != NB_SPLIT) return "precision must be NB_FP64 or NB_SPLIT";
    if (p->jchunk < 0 || p->jchunk > (1 << 20) || (p->jchunk % nb::kItemTile) != 0)
        return "jchunk must be a multiple of 64 in [0, 2^20] (0 = default)";
    if (p->items_per_job < 0 || p->items_per_job > (1 << 14))
        return "items_per_job must be in [0, 16384] (0 = default)";
    if (p->chunk_tile < 0 || p->chunk_tile > 64 || p->chunk_wide < 0 || p->chunk_wide > 64 ||
        p->chunk_direct < 0 || p->chunk_direct > 64)
        return "chunk_tile, chunk_wide and chunk_direct must be in [0, 64] (0 = default)";
    if (p->partial_slots < 0) return "partial_slots must be >= 0";
    return nullptr;
}

// Launches of one evaluation over the jobs in `list` (n_list entries, device array)
// whose n_act is in j_nact, then the finishing pass in `mode`. No host work between.
// planned: the plan of this evaluation is already built.
nb_status b_eval_finish(nb_batch *b, const int32_t *list, int n_list, int mode, int count, bool planned = false)
{
    const bool split = b->p.precision == NB_SPLIT;
    const int L = b->p.dt_max_log2 - b->p.dt_min_log2;
    if (!planned)
        hipLaunchKernelGGL(nb::k_plan, dim3(1), dim3(nb::kPlanBS), 0, b->st, b->P, list, n_list, b->split_cfg,
                           count);
    if (split) {
        const float e2 = (float)(b->p.eps * b->p.eps);
        hipLaunchKernelGGL(nb::k_beval_split, dim3(b->eval_grid), dim3(64), 0, b->st, b->P, e2);
    } else {
        const double e2 = b->p.eps * b->p.eps;
        hipLaunchKernelGGL(nb::k_beval_f64, dim3(b->eval_grid), dim3(64), 0, b->st, b->P, e2);
    }
    hipLaunchKernelGGL(nb::k_bfinish, dim3(b->finish_grid), dim3(256), 0, b->st, b->P, b->cap, mode,
                       ldexp(1.0, b->p.dt_min_log2), b->p.eta, b->p.eta_init, b->p.dt_max_log2, L);
    B_HIP(b, hipGetLastError());
    return NB_OK;
}

// One block step of every job in the batch, enqueued without waiting.
// The job list to the device when it changed since the last upload.
nb_status b_upload_jobs(nb_batch *b)
{
    if (b->jobs_dirty) {
        b->njobs = 0;
        b->npblk = 0;
        for (int k = 0; k < b->p.max_jobs; ++k)
            if (b->alive[k]) {
                b->h_jobs[b->njobs++] = k;
                for (int64_t base = 0; base < b->n[k]; base += nb::kPlanBS)
                    b->h_pblk[b->npblk++] = make_int2(k, (int)base);
            }
        if (b->njobs > 0) {
            B_HIP(b, hipMemcpyAsync(b->d_jobs, b->h_jobs, 4 * (size_t)b->njobs, hipMemcpyHostToDevice, b->st));
            B_HIP(b, hipMemcpyAsync(b->P.pblk, b->h_pblk, 8 * (size_t)b->npblk, hipMemcpyHostToDevice, b->st));
        }
        b->jobs_dirty = false;
        b->graph_valid = false;  // the captured step launches a grid per listed job
    }
    return NB_OK;
}

// The kernels of one batch step (the job list already on the device).
nb_status b_launch_step(nb_batch *b)
{
    if (b->njobs == 0)
        return NB_OK;
    const bool split = b->p.precision == NB_SPLIT;
    hipLaunchKernelGGL(nb::k_bact, dim3(b->njobs), dim3(nb::kBS), 0, b->st, b->P, (const int32_t *)b->d_jobs,
                       b->p.dt_max_log2 - b->p.dt_min_log2);
    hipLaunchKernelGGL(nb::k_bpredict_plan, dim3(1 + b->npblk), dim3(nb::kPlanBS), 0, b->st,
                       b->P, b->cap, ldexp(1.0, b->p.dt_min_log2), (int)split, (const int32_t *)b->d_jobs,
                       b->njobs, b->split_cfg);
    B_HIP(b, hipGetLastError());
    return b_eval_finish(b, b->d_jobs, b->njobs, nb::kStep, 1, true);
}

nb_status b_enqueue_step(nb_batch *b)
{
    nb_status s = b_upload_jobs(b);
    return s ? s : b_launch_step(b);
}

void b_drop_graph(nb_batch *b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->gexec[k])
            (void)hipGraphExecDestroy(b->gexec[k]);
        if (b->graph[k])
            (void)hipGraphDestroy(b->graph[k]);
        b->gexec[k] = nullptr;
        b->graph[k] = nullptr;
    }
    b->graph_valid = false;
}

// Steps per replay of the larger graph: back-to-back replays of one graph leave a
// gap of about 13 us between them, the launches inside one graph a few us.
constexpr int kGraphSteps = 8;

// Capture batch steps as graphs, replayed by multi-step calls: one step and
// kGraphSteps steps (the launches carry no per-step arguments: every size comes from
// device memory). No memset or copy is captured. Returns false (and the caller
// launches directly) when the stream cannot be captured, e.g. the null stream.
bool b_capture_step(nb_batch *b)
{
    b_drop_graph(b);
    if (!b->st || b->no_graph)
        return false;
    for (int k = 0; k < 2; ++k) {
        if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            b_drop_graph(b);
            b->no_graph = true;
            return false;
        }
        nb_status s = NB_OK;
        for (int r = 0; r < (k ? kGraphSteps : 1) && s == NB_OK; ++r)
            s = b_launch_step(b);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->st, &g);
        b->graph[k] = g;
        if (s != NB_OK || e != hipSuccess || !g ||
            hipGraphInstantiate(&b->gexec[k], g, nullptr, nullptr, 0) != hipSuccess) {
            b->gexec[k] = nullptr;
            (void)hipGetLastError();
            b_drop_graph(b);
            b->no_graph = true;
            return false;
        }
    }
    b->graph_valid = true;
    return true;
}

// Job table and step header to the host (one wait).
nb_status b_fetch(nb_batch *b)
{
    const size_t J = (size_t)b->p.max_jobs;
    B_HIP(b, hipMemcpyAsync(b->h_jobblk, b->P.j_nact, 20 * J, hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipMemcpyAsync(b->h_hdr, b->P.hdr, sizeof(nb::StepHdr), hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipStreamSynchronize(b->st));
    if (b->h_hdr->overflow)
        return bfail(b, NB_ERR_STATE, "partial-sum buffer overflow (%lld slots needed)",
                     (long long)b->h_hdr->pslots);
    return NB_OK;
}

void b_outputs(nb_batch *b, int64_t *h_n_act, int64_t *h_tick_next, int32_t *h_job_err)
{
    for (int k = 0; k < b->p.max_jobs; ++k) {
        const bool live = b->alive[k];
        if (h_n_act) h_n_act[k] = live ? b->h_nact()[k] : 0;
        if (h_tick_next) h_tick_next[k] = live ? b->h_tnext()[k] : 0;
        if (h_job_err) h_job_err[k] = live ? b->h_err()[k] : 0;
    }
}

}  // namespace

extern "C" {

nb_status nb_batch_workspace_bytes(const nb_batch_params *p, size_t *h_bytes)
{
    if (!h_bytes || b_check_params(p))
        return NB_ERR_ARG;
    Pool P{};
    int32_t *dj, *d1;
    *h_bytes = b_layout(p, &P, &dj, &d1, nullptr);
    return NB_OK;
}

nb_status nb_batch_create(const nb_batch_params *p, void *d_workspace, size_t bytes, nb_batch **out)
{
    if (!out)
        return NB_ERR_ARG;
    *out = nullptr;
    if (b_check_params(p) || !d_workspace || ((uintptr_t)d_workspace & 255))
        return NB_ERR_ARG;
    Pool P{};
    int32_t *dj, *d1;
    if (bytes < b_layout(p, &P, &dj, &d1, nullptr))
        return NB_ERR_SPACE;
    nb_batch *b = new (std::nothrow) nb_batch();
    if (!b)
        return NB_ERR_SPACE;
    b->p = *p;
    b->st = (hipStream_t)p->stream;
    b->cap = p->capacity;
    b->partial_slots = b_partial_slots(p);
    b->split_cfg = b_split_cfg(p);
    b_layout(p, &b->P, &b->d_jobs, &b->d_one, (char *)d_workspace);
    const size_t J = (size_t)p->max_jobs;
    b->off.assign(J, 0);
    b->n.assign(J, 0);
    b->tend.assign(J, 0);
    b->alive.assign(J, 0);
    b->free_ranges.push_back({0, p->capacity});
    b->jobs_dirty = true;
    // persistent evaluation: as many waves as can be resident on the device
    int dev = 0, cus = 0, per = 0, fin = 0;
    const bool sp = p->precision == NB_SPLIT;
    bool ok = hipGetDevice(&dev) == hipSuccess &&
              hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
              hipOccupancyMaxActiveBlocksPerMultiprocessor(&fin, nb::k_bfinish, 256, 0) == hipSuccess &&
              (sp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, nb::k_beval_split, 64, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, nb::k_beval_f64, 64, 0)) == hipSuccess;
    b->eval_grid = std::max(1, cus * std::max(1, per));
    b->finish_grid = std::max(1, cus * std::max(1, fin));
    ok = ok && hipHostMalloc((void **)&b->h_scalar, 64, 0) == hipSuccess &&
         hipHostMalloc((void **)&b->h_jobblk, 20 * J, 0) == hipSuccess &&
         hipHostMalloc((void **)&b->h_hdr, sizeof(nb::StepHdr), 0) == hipSuccess &&
         hipHostMalloc((void **)&b->h_jobs, 4 * J, 0) == hipSuccess &&
         hipHostMalloc((void **)&b->h_pblk, 8 * (size_t)b_pblk_max(p), 0) == hipSuccess &&
         hipHostMalloc((void **)&b->h_status, sizeof(nb::Status), 0) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(nb::k_hdr_reset, dim3(1), dim3(64), 0, b->st, b->P);
        ok = hipGetLastError() == hipSuccess &&
             nb::launch_fill_i32(b->P.j_err, 0, J, b->st) == hipSuccess &&
             nb::launch_fill_i64(b->P.j_nact, 0, J, b->st) == hipSuccess &&
             nb::launch_fill_i32((int32_t *)b->P.status, 0, sizeof(nb::Status) / 4, b->st) == hipSuccess &&
             b_fetch(b) == NB_OK;  // the host copies start current
    }
    if (!ok) {
        nb_batch_destroy(b);
        return NB_ERR_DEVICE;
    }
    *out = b;
    return NB_OK;
}

void nb_batch_destroy(nb_batch *b)
{
    if (!b)
        return;
    (void)hipStreamSynchronize(b->st);
    b_drop_graph(b);
    for (void *q : {(void *)b->h_scalar, (void *)b->h_jobblk, (void *)b->h_hdr, (void *)b->h_jobs,
                    (void *)b->h_pblk, (void *)b->h_status})
        if (q)
            (void)hipHostFree(q);
    delete b;
}

const char *nb_batch_last_error(const nb_batch *b) { return b ? b->msg : "null batch"; }

nb_status nb_batch_add(nb_batch *b, int64_t n, const nb_state *src, int64_t tick0, int64_t tick_end,
                       int32_t *h_job)
{
    if (!b)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    if (!h_job || !src || !src->m || !src->x || !src->v || n < 1)
        return bfail(b, NB_ERR_ARG, "need n >= 1, m, x, v and h_job");
    if (tick_end < tick0)
        return bfail(b, NB_ERR_ARG, "tick_end < tick0");
    // admission: a free job slot and a free contiguous range of n bodies (first fit)
    int job = -1;
    for (int k = 0; k < b->p.max_jobs; ++k)
        if (!b->alive[k]) { job = k; break; }
    if (job < 0)
        return bfail(b, NB_ERR_SPACE, "no free job slot");
    size_t r = 0;
    for (; r < b->free_ranges.size(); ++r)
        if (b->free_ranges[r].second >= n)
            break;
    if (r == b->free_ranges.size())
        return bfail(b, NB_ERR_SPACE, "no free range of %lld bodies", (long long)n);
    const int64_t off = b->free_ranges[r].first;
    const bool synced = !src->tick;
    b->jobs_dirty = true;
    // load the state; the pinned scalars are free (every call ends with a wait)
    b->h_scalar[0] = tick_end;
    reinterpret_cast<int32_t *>(b->h_scalar + 1)[0] = job;
    hipLaunchKernelGGL(nb::k_bload, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap, off, n,
                       src->m, src->x, src->v, src->a, src->j, src->s, src->c, src->a4n, src->a5n,
                       src->tick, src->level, tick0);
    hipLaunchKernelGGL(nb::k_bjob_init, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, job, off, n,
                       tick0);
    B_HIP(b, hipGetLastError());
    B_HIP(b, hipMemcpyAsync(b->P.j_tend + job, b->h_scalar, 8, hipMemcpyHostToDevice, b->st));
    B_HIP(b, hipMemcpyAsync(b->d_one, b->h_scalar + 1, 4, hipMemcpyHostToDevice, b->st));
    b->off[job] = off;
    b->n[job] = n;
    b->tend[job] = tick_end;
    nb_status s = NB_OK;
    if (synced) {
        // Hermite start-up of this job alone: every body evaluated twice (the second
        // time with the first pass's accelerations in the records), then levels
        const bool split = b->p.precision == NB_SPLIT;
        hipLaunchKernelGGL(nb::k_bpredict_range, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap,
                           off, n, tick0, ldexp(1.0, b->p.dt_min_log2), (int)split);
        s = b_eval_finish(b, b->d_one, 1, nb::kStartA, 0);
        if (!s)
            s = b_eval_finish(b, b->d_one, 1, nb::kStartB, 0);
    }
    if (!s)
        s = b_fetch(b);
    if (s) {
        // leave the range and the job slot unclaimed, so no later step touches them
        (void)nb::launch_fill_i64(b->P.j_nact + job, 0, 1, b->st);
        (void)hipStreamSynchronize(b->st);
        return s;
    }
    // commit the reservation
    b->free_ranges[r].first += n;
    b->free_ranges[r].second -= n;
    if (b->free_ranges[r].second == 0)
        b->free_ranges.erase(b->free_ranges.begin() + r);
    b->alive[job] = 1;
    *h_job = job;
    return NB_OK;
}

nb_status nb_batch_remove(nb_batch *b, int32_t job)
{
    if (!b)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    if (job < 0 || job >= b->p.max_jobs || !b->alive[job])
        return bfail(b, NB_ERR_ARG, "job %d is not in the batch", job);
    b->jobs_dirty = true;
    B_HIP(b, nb::launch_fill_i64(b->P.j_nact + job, 0, 1, b->st));
    B_HIP(b, hipGetLastError());
    B_HIP(b, hipStreamSynchronize(b->st));
    // return the range and merge neighbours
    b->free_ranges.push_back({b->off[job], b->n[job]});
    std::sort(b->free_ranges.begin(), b->free_ranges.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (auto &fr : b->free_ranges) {
        if (!merged.empty() && merged.back().first + merged.back().second == fr.first)
            merged.back().second += fr.second;
        else
            merged.push_back(fr);
    }
    b->free_ranges.swap(merged);
    b->alive[job] = 0;
    b->n[job] = 0;
    return NB_OK;
}

nb_status nb_batch_step(nb_batch *b, int64_t *h_n_act, int64_t *h_tick_next, int32_t *h_job_err,
                        int64_t *h_interactions)
{
    if (!b)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    nb_status s;
    const int64_t before = b->h_hdr->inter;  // host copy is current: every call ends with a fetch
    if ((s = b_enqueue_step(b)) || (s = b_fetch(b)))
        return s;
    b_outputs(b, h_n_act, h_tick_next, h_job_err);
    if (h_interactions)
        *h_interactions = b->h_hdr->inter - before;
    return NB_OK;
}

nb_status nb_batch_run(nb_batch *b, int32_t steps, int64_t *h_n_act, int64_t *h_tick_next,
                       int32_t *h_job_err, int64_t *h_interactions, int64_t *h_steps)
{
    if (!b)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    if (steps < 1)
        return bfail(b, NB_ERR_ARG, "steps must be >= 1");
    nb_status s;
    const int64_t inter0 = b->h_hdr->inter, steps0 = b->h_hdr->steps;
    if ((s = b_upload_jobs(b)))
        return s;
    if (b->njobs > 0 && steps > 1 && (b->graph_valid || b_capture_step(b))) {
        for (int k = 0; k < steps / kGraphSteps; ++k)
            B_HIP(b, hipGraphLaunch(b->gexec[1], b->st));
        for (int k = 0; k < steps % kGraphSteps; ++k)
            B_HIP(b, hipGraphLaunch(b->gexec[0], b->st));
    } else {
        for (int k = 0; k < steps; ++k)
            if ((s = b_launch_step(b)))
                return s;
    }
    if ((s = b_fetch(b)))
        return s;
    b_outputs(b, h_n_act, h_tick_next, h_job_err);
    if (h_interactions)
        *h_interactions = b->h_hdr->inter - inter0;
    if (h_steps)
        *h_steps = b->h_hdr->steps - steps0;
    return NB_OK;
}

nb_status nb_batch_get(nb_batch *b, int32_t job, const nb_state *dst)
{
    if (!b || !dst)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    if (job < 0 || job >= b->p.max_jobs || !b->alive[job])
        return bfail(b, NB_ERR_ARG, "job %d is not in the batch", job);
    const int64_t n = b->n[job];
    hipLaunchKernelGGL(nb::k_bstore, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap, b->off[job], n,
                       dst->m, dst->x, dst->v, dst->a, dst->j, dst->s, dst->c, dst->a4n, dst->a5n, dst->phi,
                       dst->tick, dst->level);
    B_HIP(b, hipGetLastError());
    B_HIP(b, hipStreamSynchronize(b->st));
    return NB_OK;
}

nb_status nb_batch_energy(nb_batch *b, int32_t job, int64_t tick, double *h_ekin, double *h_epot)
{
    if (!b || !h_ekin || !h_epot)
        return NB_ERR_ARG;
    b->msg[0] = 0;
    if (job < 0 || job >= b->p.max_jobs || !b->alive[job])
        return bfail(b, NB_ERR_ARG, "job %d is not in the batch", job);
    const int64_t n = b->n[job], off = b->off[job];
    // predicting into the records is harmless: every step predicts its jobs again
    hipLaunchKernelGGL(nb::k_bpredict_range, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap, off,
                       n, tick, ldexp(1.0, b->p.dt_min_log2), 0);
    B_HIP(b, hipGetLastError());
    // the single-system energy kernels on a view of this job's records
    nb::Arrays A{};
    A.jrec = b->P.jrec + off * nb::kRecD;
    A.part = b->P.part;
    A.en_bsum = b->P.en_bsum;
    A.status = b->P.status;
    B_HIP(b, nb::launch_energy(A, n, b->p.eps, b->partial_slots, b->st));
    B_HIP(b, hipMemcpyAsync(b->h_status, b->P.status, sizeof(nb::Status), hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipStreamSynchronize(b->st));
    *h_ekin = b->h_status->ekin;
    *h_epot = b->h_status->epot;
    return NB_OK;
}

nb_status nb_batch_info(const nb_batch *b, int32_t job, int64_t *h_offset, int64_t *h_n)
{
    if (!b || job < 0 || job >= b->p.max_jobs || !b->alive[job])
        return NB_ERR_ARG;
    if (h_offset) *h_offset = b->off[job];
    if (h_n) *h_n = b->n[job];
    return NB_OK;
}

}  // extern "C"
