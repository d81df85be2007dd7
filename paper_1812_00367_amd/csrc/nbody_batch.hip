// nbody_batch.hip -- many independent N-body systems ("jobs") of uneven size in one
// workspace, advanced together: every batch step gives each job its own next block
// step (its own block time and active set), with one launch per kernel for all jobs.
//
// Pool layout: all jobs' bodies live in one pool of `capacity` bodies (job j owns
// the contiguous range [off_j, off_j + n_j)); vectors are [3][capacity]
// structure-of-arrays, the j-records are the same 80-byte (and 64-byte split)
// records as the single-system path. The evaluation of a batch step is one launch
// over a list of work items (job, 64-body active tile, j-chunk of `jchunk` bodies);
// each job's partial sums are added in a fixed order afterwards. A job's arithmetic
// therefore depends only on its own data and on jchunk, never on the other jobs:
// its results are bitwise the same alone and in any mix.
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

constexpr int kItemTile = 64;  // active bodies per work item (one wave, one per lane)

struct Pool {
    double *m, *x, *v, *a, *j, *s, *c, *a4n, *a5n, *phi;
    int64_t *tick;
    int32_t *level;
    int32_t *body_job;  // job id of every pool slot, -1 when free
    double *jrec;
    float *jrec32;
    double *evalbuf;    // [10][n_act_j] at 10 * off_j for job j
    int32_t *act;       // job j's active list (pool indices) at off_j
    double *part;
    // job table
    int64_t *j_off, *j_n, *j_nact, *j_tnext, *j_tend;
    int32_t *j_err;
    // per-launch group description (uploaded each batch step)
    int32_t *items;     // [items_cap][4] = job, i-tile, split, group entry
    int64_t *g_desc;    // [5][group_cap]: job, pbase, rbase (10 n_act prefix), nbase (n_act prefix), S
    int64_t *g_desc2;   // the same for the corrector and step levels
    double *en_bsum;
    Status *status;
};

// -------------------------------------------------------- active selection ----
// One workgroup per listed job: tick_next = min over its bodies of t + dt, then the
// bodies due at tick_next in ascending order into act[off ...]; n_act = 0 when
// tick_next is beyond the job's end time.
constexpr int kBS = 256;

__global__ __launch_bounds__(kBS) void k_bact(Pool P, const int32_t *__restrict__ jobs, int L)
{
    __shared__ int64_t red[kBS / 64];
    __shared__ int wc[kBS / 64];
    const int job = jobs[blockIdx.x];
    const int64_t off = P.j_off[job], n = P.j_n[job];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t mn = INT64_MAX;
    bool badlevel = false;
    for (int64_t k = threadIdx.x; k < n; k += kBS) {
        int lv = P.level[off + k];
        if (lv < 0 || lv > L) {
            badlevel = true;
            lv = L;
        }
        const int64_t e = P.tick[off + k] + ((int64_t)1 << (L - lv));
        mn = e < mn ? e : mn;
    }
    if (badlevel)
        P.j_err[job] = kJobLevel;
    mn = wave_min_i64(mn);
    if (lane == 0)
        red[wave] = mn;
    __syncthreads();
    int64_t tn = red[0];
    for (int w = 1; w < kBS / 64; ++w)
        tn = red[w] < tn ? red[w] : tn;
    const bool beyond = tn > P.j_tend[job];
    int64_t base = 0;
    if (!beyond) {
        for (int64_t r0 = 0; r0 < n; r0 += kBS) {
            const int64_t k = r0 + threadIdx.x;
            bool due = false;
            if (k < n) {
                int lv = P.level[off + k];
                lv = (lv < 0 || lv > L) ? L : lv;
                due = P.tick[off + k] + ((int64_t)1 << (L - lv)) == tn;
            }
            const unsigned long long mask = __ballot(due);
            if (lane == 0)
                wc[wave] = __popcll(mask);
            __syncthreads();
            int before = 0, tot = 0;
            for (int w = 0; w < kBS / 64; ++w) {
                before += (w < wave) ? wc[w] : 0;
                tot += wc[w];
            }
            if (due)
                P.act[off + base + before + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)(off + k);
            base += tot;
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        P.j_tnext[job] = tn;
        P.j_nact[job] = beyond ? 0 : base;
    }
}

// --------------------------------------------------------------- prediction ----
// Every body of a job that steps (n_act > 0) to its job's block time.
__global__ __launch_bounds__(256) void k_bpredict(Pool P, int64_t cap, double tick_size, int split)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap)
        return;
    const int job = P.body_job[i];
    if (job < 0 || P.j_nact[job] == 0)
        return;
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
// One wave per work item (job, i-tile, split): the item's 64 active bodies against
// the job's j-chunk, partial sums to part[pbase + (s * 10 + c) * n_act + q].
template <bool SPLIT>
__global__ __launch_bounds__(64) void k_beval(Pool P, const int32_t *__restrict__ items,
                                              const int64_t *__restrict__ gd, int ngroup, int jchunk,
                                              double eps2)
{
    constexpr int BS = 64;
    const int4 it = reinterpret_cast<const int4 *>(items)[blockIdx.x];
    const int job = it.x, ib = it.y, sp = it.z, gi = it.w;
    const int64_t off = P.j_off[job], n = P.j_n[job];
    const int na = (int)P.j_nact[job];
    const int64_t pbase = gd[1 * ngroup + gi];
    const int jbeg = (int)(off + (int64_t)sp * jchunk);
    const int jend = (int)min(off + n, (int64_t)jbeg + jchunk);
    const int32_t *act = P.act + off;
    bool bad;
    int lo, hi;
    if (SPLIT) {
        __shared__ float4 lds[2][kItemTile * 4];
        I32 b[1];
        load_i_split<1, BS>(P.jrec32, act, na, ib * BS, (int)off, (int)(off + n), b, lo, hi, bad);
        tiles_split<1, 1, kItemTile>(P.jrec32, jbeg, jend, b, lo, hi, (float)eps2, lds);
        const int slot = ib * BS + (int)threadIdx.x;
        if (slot < na)
            for (int c = 0; c < 10; ++c)
                P.part[pbase + ((int64_t)sp * 10 + c) * na + slot] = b[0].acc[c];
    } else {
        __shared__ double2 lds[2][kItemTile * 5];
        I64 b[1];
        load_i_f64<1, BS>(P.jrec, act, na, ib * BS, (int)off, (int)(off + n), b, lo, hi, bad);
        tiles_f64<1, 1, kItemTile>(P.jrec, jbeg, jend, b, lo, hi, eps2, lds);
        const int slot = ib * BS + (int)threadIdx.x;
        if (slot < na)
            for (int c = 0; c < 10; ++c)
                P.part[pbase + ((int64_t)sp * 10 + c) * na + slot] = b[0].acc[c];
    }
    if (bad)
        P.j_err[job] = kJobLevel;
}

// Locate the group entry g with prefix[g] <= e < prefix[g + 1] (prefix ascending,
// prefix[0] = 0, ngroup entries).
__device__ __forceinline__ int group_of(const int64_t *__restrict__ prefix, int ngroup, int64_t e)
{
    int lo = 0, hi = ngroup - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Fixed-order sum over each job's S splits into evalbuf[10 off + c n_act + q].
__global__ __launch_bounds__(256) void k_breduce(Pool P, const int64_t *__restrict__ gd, int ngroup,
                                                 int64_t total)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total)
        return;
    const int g = group_of(gd + 2 * ngroup, ngroup, e);
    const int job = (int)gd[g];
    const int64_t pbase = gd[1 * ngroup + g], local = e - gd[2 * ngroup + g];
    const int S = (int)gd[4 * ngroup + g];
    const int64_t na = P.j_nact[job];
    double acc = 0.0;
    for (int s = 0; s < S; ++s)
        acc += P.part[pbase + (int64_t)s * 10 * na + local];
    P.evalbuf[10 * P.j_off[job] + local] = acc;
}

// -------------------------------------------------- corrector and step levels ----
__global__ __launch_bounds__(256) void k_bcorrect(Pool P, int64_t cap, const int64_t *__restrict__ gd,
                                                  int ngroup, int64_t total, double tick_size)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total)
        return;
    const int g = group_of(gd + 3 * ngroup, ngroup, e);
    const int job = (int)gd[g];
    const int64_t q = e - gd[3 * ngroup + g], off = P.j_off[job], na = P.j_nact[job];
    const int64_t i = P.act[off + q];
    const int64_t tn = P.j_tnext[job], ti = P.tick[i];
    if (ti >= tn) {
        P.j_err[job] = kJobLevel;
        return;
    }
    const double *ev = P.evalbuf + 10 * off + q;
    const bool ok = correct_body(P.x, P.v, P.a, P.j, P.s, P.c, P.a4n, P.a5n, (size_t)cap, (size_t)i,
                                 ev, (size_t)na, (double)(tn - ti) * tick_size);
    P.phi[i] = ev[9 * na];
    P.tick[i] = tn;
    if (!ok)
        P.j_err[job] = kJobNumeric;
}

__global__ __launch_bounds__(256) void k_blevels(Pool P, int64_t cap, const int64_t *__restrict__ gd,
                                                 int ngroup, int64_t total, int init, double eta,
                                                 double eta_init, int dt_max_log2, int L)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total)
        return;
    const int g = group_of(gd + 3 * ngroup, ngroup, e);
    const int job = (int)gd[g];
    const int64_t i = P.act[P.j_off[job] + (e - gd[3 * ngroup + g])];
    bool dtmin;
    P.level[i] = level_for_body(P.a, P.j, P.s, P.c, P.a4n, P.a5n, (size_t)cap, (size_t)i, P.tick[i],
                                P.level[i], init, eta, eta_init, dt_max_log2, L, &dtmin);
    if (dtmin)
        P.j_err[job] = kJobDtMin;
}

// ------------------------------------------------------------- start-up ----
// Active list = every body of the job; store the start-up evaluation; copy the
// first evaluation's accelerations into the predicted records.
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
    }
    if (k < n) {
        P.act[off + k] = (int32_t)(off + k);
        P.body_job[off + k] = job;
    }
}

__global__ __launch_bounds__(256) void k_bacc_to_jrec(Pool P, int64_t off, int64_t n, int split)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = off + k;
    for (int c = 0; c < 3; ++c) {
        const double a = P.evalbuf[10 * off + (int64_t)c * n + k];
        P.jrec[i * kRecD + 6 + c] = a;
        if (split)
            P.jrec32[i * kRecF + 12 + c] = (float)a;
    }
}

__global__ __launch_bounds__(256) void k_bstart_store(Pool P, int64_t cap, int64_t off, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = off + k;
    const double *e = P.evalbuf + 10 * off;
    for (int c = 0; c < 3; ++c) {
        P.a[c * cap + i] = e[(0 + c) * n + k];
        P.j[c * cap + i] = e[(3 + c) * n + k];
        P.s[c * cap + i] = e[(6 + c) * n + k];
        P.c[c * cap + i] = 0.0;
    }
    P.phi[i] = e[9 * n + k];
    P.a4n[i] = 0.0;
    P.a5n[i] = 0.0;
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

__global__ __launch_bounds__(256) void k_bfree(Pool P, int64_t off, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n)
        P.body_job[off + k] = -1;
}

unsigned nblk(int64_t count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace
}  // namespace nb

using nb::Pool;

struct nb_batch {
    nb_batch_params p;
    hipStream_t st;
    Pool P;
    int64_t cap, items_cap, group_cap, partial_slots;
    char msg[512];
    // host job table
    std::vector<int64_t> off, n, tend;
    std::vector<char> alive;
    std::vector<std::pair<int64_t, int64_t>> free_ranges;  // (offset, length), sorted
    // pinned host staging
    int32_t *h_items;
    int64_t *h_desc, *h_desc2;
    int64_t *h_scalar;
    int64_t *h_nact, *h_tnext;
    int32_t *h_err;
    int32_t *h_jobs;
    int32_t *d_jobs;
    nb::Status *h_status;
    hipEvent_t staged;  // recorded after the last copy out of h_items / h_desc
    bool staged_valid, has_event;
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int64_t kItemsCap = (int64_t)1 << 20;

int64_t b_partial_slots(const nb_batch_params *p)
{
    if (p->partial_slots > 0)
        return p->partial_slots;
    const int64_t a = 4 * p->capacity, b = (int64_t)1 << 22;
    return a > b ? a : b;
}

int b_jchunk(const nb_batch_params *p) { return p->jchunk > 0 ? p->jchunk : 1024; }

// device workspace layout; returns bytes (base may be null to measure)
size_t b_layout(const nb_batch_params *p, Pool *P, int32_t **d_jobs, int64_t *items_cap,
                int64_t *group_cap, char *base)
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
    // work items per launch (a batch step with more is split over several launches;
    // one job's full evaluation must fit on its own)
    *items_cap = kItemsCap;
    *group_cap = (int64_t)J;
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
    P->body_job = (int32_t *)take(4 * cap);
    P->jrec = (double *)take(8 * nb::kRecD * cap);
    P->jrec32 = split ? (float *)take(4 * nb::kRecF * cap) : nullptr;
    P->evalbuf = (double *)take(80 * cap);
    P->act = (int32_t *)take(4 * cap);
    P->part = (double *)take(80 * (size_t)ps);
    P->j_off = (int64_t *)take(8 * J);
    P->j_n = (int64_t *)take(8 * J);
    P->j_nact = (int64_t *)take(8 * J);
    P->j_tnext = (int64_t *)take(8 * J);
    P->j_tend = (int64_t *)take(8 * J);
    P->j_err = (int32_t *)take(4 * J);
    P->items = (int32_t *)take(16 * (size_t)*items_cap);
    P->g_desc = (int64_t *)take(8 * 5 * (size_t)*group_cap);
    P->g_desc2 = (int64_t *)take(8 * 5 * (size_t)*group_cap);
    P->en_bsum = (double *)take(16 * (size_t)nb::en_blocks(p->capacity));
    P->status = (nb::Status *)take(sizeof(nb::Status));
    *d_jobs = (int32_t *)take(4 * J);
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
    if (p->max_jobs < 1 || p->max_jobs > (1 << 20)) return "max_jobs must be in [1, 2^20]";
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return "eps must be finite and >= 0";
    if (!(p->eta > 0.0) || !isfinite(p->eta) || !(p->eta_init > 0.0) || !isfinite(p->eta_init))
        return "eta and eta_init must be finite and > 0";
    if (p->dt_max_log2 > 100 || p->dt_min_log2 < -200) return "dt_max_log2 <= 100 and dt_min_log2 >= -200";
    const int L = p->dt_max_log2 - p->dt_min_log2;
    if (L < 0 || L > 62) return "need 0 <= dt_max_log2 - dt_min_log2 <= 62";
    if (p->precision != NB_FP64 && p->precision != NB_SPLIT) return "precision must be NB_FP64 or NB_SPLIT";
    if (p->jchunk < 0 || (p->jchunk % nb::kItemTile) != 0) return "jchunk must be a multiple of 64 (0 = default)";
    if (p->reserved != 0) return "reserved must be 0";
    if (p->partial_slots < 0) return "partial_slots must be >= 0";
    return nullptr;
}

// Evaluate the active sets of `group` (jobs with n_act > 0, in the host arrays
// b->h_nact), in launches that fit the partial and item buffers; results land in
// each job's evaluation block. Host arrays hold n_act of every listed job.
nb_status b_evaluate(nb_batch *b, const std::vector<int> &group)
{
    const int jchunk = b_jchunk(&b->p);
    const int64_t ps = b->partial_slots;
    const double eps2 = b->p.eps * b->p.eps;
    size_t k = 0;
    while (k < group.size()) {
        // take jobs while the items and partials fit
        int64_t nitems = 0, pslots = 0;
        size_t e = k;
        std::vector<int> gj;
        while (e < group.size()) {
            const int job = group[e];
            const int64_t na = b->h_nact[job];
            const int64_t S = (b->n[job] + jchunk - 1) / jchunk;
            const int64_t it = (na + nb::kItemTile - 1) / nb::kItemTile * S;
            if (S * na > ps)
                return bfail(b, NB_ERR_SPACE, "job %d needs %lld partial slots (capacity %lld)", job,
                             (long long)(S * na), (long long)ps);
            if (!gj.empty() && (nitems + it > b->items_cap || pslots + S * na > ps ||
                                (int64_t)gj.size() >= b->group_cap))
                break;
            if (it > b->items_cap)
                return bfail(b, NB_ERR_SPACE, "job %d needs %lld work items", job, (long long)it);
            gj.push_back(job);
            nitems += it;
            pslots += S * na;
            ++e;
        }
        const int ng = (int)gj.size();
        // the previous launch's copies out of the staging buffers must have run
        if (b->staged_valid)
            B_HIP(b, hipEventSynchronize(b->staged));
        int64_t pbase = 0, rbase = 0, nbase = 0, w = 0;
        for (int g = 0; g < ng; ++g) {
            const int job = gj[g];
            const int64_t na = b->h_nact[job];
            const int64_t S = (b->n[job] + jchunk - 1) / jchunk;
            b->h_desc[0 * ng + g] = job;
            b->h_desc[1 * ng + g] = pbase;
            b->h_desc[2 * ng + g] = rbase;
            b->h_desc[3 * ng + g] = nbase;
            b->h_desc[4 * ng + g] = S;
            const int64_t tiles = (na + nb::kItemTile - 1) / nb::kItemTile;
            for (int64_t t = 0; t < tiles; ++t)
                for (int64_t s = 0; s < S; ++s) {
                    int32_t *it = b->h_items + 4 * w++;
                    it[0] = job;
                    it[1] = (int32_t)t;
                    it[2] = (int32_t)s;
                    it[3] = g;
                }
            pbase += S * 10 * na;
            rbase += 10 * na;
            nbase += na;
        }
        B_HIP(b, hipMemcpyAsync(b->P.items, b->h_items, 16 * (size_t)w, hipMemcpyHostToDevice, b->st));
        B_HIP(b, hipMemcpyAsync(b->P.g_desc, b->h_desc, 8 * 5 * (size_t)ng, hipMemcpyHostToDevice, b->st));
        B_HIP(b, hipEventRecord(b->staged, b->st));
        b->staged_valid = true;
        if (b->p.precision == NB_SPLIT)
            hipLaunchKernelGGL(nb::k_beval<true>, dim3((unsigned)w), dim3(64), 0, b->st, b->P,
                               (const int32_t *)b->P.items, (const int64_t *)b->P.g_desc, ng, jchunk, eps2);
        else
            hipLaunchKernelGGL(nb::k_beval<false>, dim3((unsigned)w), dim3(64), 0, b->st, b->P,
                               (const int32_t *)b->P.items, (const int64_t *)b->P.g_desc, ng, jchunk, eps2);
        B_HIP(b, hipGetLastError());
        hipLaunchKernelGGL(nb::k_breduce, dim3(nb::nblk(rbase, 256)), dim3(256), 0, b->st, b->P,
                           (const int64_t *)b->P.g_desc, ng, rbase);
        B_HIP(b, hipGetLastError());
        k = e;
    }
    return NB_OK;
}

// corrector + levels for a group described in g_desc (already uploaded)
nb_status b_correct_levels(nb_batch *b, const std::vector<int> &group, int init)
{
    // corrector and levels are launched once per group of at most group_cap jobs
    const double tick_size = ldexp(1.0, b->p.dt_min_log2);
    const int L = b->p.dt_max_log2 - b->p.dt_min_log2;
    size_t k = 0;
    while (k < group.size()) {
        const int ng = (int)std::min<size_t>(group.size() - k, (size_t)b->group_cap);
        int64_t nbase = 0;
        for (int g = 0; g < ng; ++g) {
            const int job = group[k + g];
            b->h_desc2[0 * ng + g] = job;
            b->h_desc2[1 * ng + g] = 0;
            b->h_desc2[2 * ng + g] = 0;
            b->h_desc2[3 * ng + g] = nbase;
            b->h_desc2[4 * ng + g] = 0;
            nbase += b->h_nact[job];
        }
        B_HIP(b, hipMemcpyAsync(b->P.g_desc2, b->h_desc2, 8 * 5 * (size_t)ng, hipMemcpyHostToDevice, b->st));
        if (!init)
            hipLaunchKernelGGL(nb::k_bcorrect, dim3(nb::nblk(nbase, 256)), dim3(256), 0, b->st, b->P,
                               b->cap, (const int64_t *)b->P.g_desc2, ng, nbase, tick_size);
        hipLaunchKernelGGL(nb::k_blevels, dim3(nb::nblk(nbase, 256)), dim3(256), 0, b->st, b->P, b->cap,
                           (const int64_t *)b->P.g_desc2, ng, nbase, init, b->p.eta, b->p.eta_init,
                           b->p.dt_max_log2, L);
        B_HIP(b, hipGetLastError());
        B_HIP(b, hipStreamSynchronize(b->st));
        k += ng;
    }
    return NB_OK;
}

nb_status b_fetch_jobs(nb_batch *b)
{
    const size_t J = (size_t)b->p.max_jobs;
    B_HIP(b, hipMemcpyAsync(b->h_nact, b->P.j_nact, 8 * J, hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipMemcpyAsync(b->h_tnext, b->P.j_tnext, 8 * J, hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipMemcpyAsync(b->h_err, b->P.j_err, 4 * J, hipMemcpyDeviceToHost, b->st));
    B_HIP(b, hipStreamSynchronize(b->st));
    return NB_OK;
}

}  // namespace

extern "C" {

nb_status nb_batch_workspace_bytes(const nb_batch_params *p, size_t *h_bytes)
{
    if (!h_bytes || b_check_params(p))
        return NB_ERR_ARG;
    Pool P{};
    int32_t *dj;
    int64_t ic, gc;
    *h_bytes = b_layout(p, &P, &dj, &ic, &gc, nullptr);
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
    int32_t *dj;
    int64_t ic, gc;
    if (bytes < b_layout(p, &P, &dj, &ic, &gc, nullptr))
        return NB_ERR_SPACE;
    nb_batch *b = new (std::nothrow) nb_batch();
    if (!b)
        return NB_ERR_SPACE;
    b->p = *p;
    b->st = (hipStream_t)p->stream;
    b->cap = p->capacity;
    b->partial_slots = b_partial_slots(p);
    b_layout(p, &b->P, &b->d_jobs, &b->items_cap, &b->group_cap, (char *)d_workspace);
    const size_t J = (size_t)p->max_jobs;
    b->off.assign(J, 0);
    b->n.assign(J, 0);
    b->tend.assign(J, 0);
    b->alive.assign(J, 0);
    b->free_ranges.push_back({0, p->capacity});
    bool ok = hipHostMalloc((void **)&b->h_items, 16 * (size_t)b->items_cap, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_desc, 8 * 5 * (size_t)b->group_cap, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_desc2, 8 * 5 * (size_t)b->group_cap, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_scalar, 64, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_nact, 8 * J, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_tnext, 8 * J, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_err, 4 * J, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_jobs, 4 * J, 0) == hipSuccess &&
              hipHostMalloc((void **)&b->h_status, sizeof(nb::Status), 0) == hipSuccess &&
              hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess;
    b->has_event = ok;
    if (ok) {
        ok = nb::launch_fill_i32(b->P.body_job, -1, (size_t)b->cap, b->st) == hipSuccess &&
             nb::launch_fill_i32(b->P.j_err, 0, J, b->st) == hipSuccess &&
             nb::launch_fill_i64(b->P.j_nact, 0, J, b->st) == hipSuccess &&
             nb::launch_fill_i32((int32_t *)b->P.status, 0, sizeof(nb::Status) / 4, b->st) == hipSuccess &&
             hipStreamSynchronize(b->st) == hipSuccess;
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
    for (void *q : {(void *)b->h_items, (void *)b->h_desc, (void *)b->h_desc2, (void *)b->h_scalar,
                    (void *)b->h_nact, (void *)b->h_tnext,
                    (void *)b->h_err, (void *)b->h_jobs, (void *)b->h_status})
        if (q)
            (void)hipHostFree(q);
    if (b->has_event)
        (void)hipEventDestroy(b->staged);
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
    {
        const int64_t S = (n + b_jchunk(&b->p) - 1) / b_jchunk(&b->p);
        if ((n + nb::kItemTile - 1) / nb::kItemTile * S > b->items_cap || S * n > b->partial_slots)
            return bfail(b, NB_ERR_SPACE, "a job of %lld bodies exceeds the work-item or partial-sum "
                                          "capacity", (long long)n);
    }
    const int64_t off = b->free_ranges[r].first;
    const bool synced = !src->tick;
    // load the state
    hipLaunchKernelGGL(nb::k_bload, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap, off, n,
                       src->m, src->x, src->v, src->a, src->j, src->s, src->c, src->a4n, src->a5n,
                       src->tick, src->level, tick0);
    hipLaunchKernelGGL(nb::k_bjob_init, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, job, off, n,
                       tick0);
    B_HIP(b, hipGetLastError());
    B_HIP(b, hipStreamSynchronize(b->st));  // the pinned scalar may still be in use
    b->h_scalar[0] = tick_end;
    B_HIP(b, hipMemcpyAsync(b->P.j_tend + job, b->h_scalar, 8, hipMemcpyHostToDevice, b->st));
    b->off[job] = off;
    b->n[job] = n;
    b->tend[job] = tick_end;
    if (synced) {
        // Hermite start-up of this job alone: two evaluations of every body, then levels
        const bool split = b->p.precision == NB_SPLIT;
        const double ts = ldexp(1.0, b->p.dt_min_log2);
        std::vector<int> g{job};
        b->h_nact[job] = n;
        hipLaunchKernelGGL(nb::k_bpredict_range, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, b->cap,
                           off, n, tick0, ts, (int)split);
        nb_status s = b_evaluate(b, g);
        if (!s) {
            hipLaunchKernelGGL(nb::k_bacc_to_jrec, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, off,
                               n, (int)split);
            s = b_evaluate(b, g);
        }
        if (!s) {
            hipLaunchKernelGGL(nb::k_bstart_store, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P,
                               b->cap, off, n);
            s = hipGetLastError() == hipSuccess ? b_correct_levels(b, g, 1)
                                                : bfail(b, NB_ERR_DEVICE, "start-up launch failed");
        }
        if (s) {
            // leave the range and the job slot unclaimed, so no later step touches them
            hipLaunchKernelGGL(nb::k_bfree, dim3(nb::nblk(n, 256)), dim3(256), 0, b->st, b->P, off, n);
            (void)nb::launch_fill_i64(b->P.j_nact + job, 0, 1, b->st);
            (void)hipStreamSynchronize(b->st);
            return s;
        }
    }
    B_HIP(b, hipStreamSynchronize(b->st));
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
    hipLaunchKernelGGL(nb::k_bfree, dim3(nb::nblk(b->n[job], 256)), dim3(256), 0, b->st, b->P, b->off[job],
                       b->n[job]);
    B_HIP(b, hipGetLastError());
    B_HIP(b, hipStreamSynchronize(b->st));
    b->h_scalar[1] = 0;
    B_HIP(b, hipMemcpyAsync(b->P.j_nact + job, b->h_scalar + 1, 8, hipMemcpyHostToDevice, b->st));
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
    const int L = b->p.dt_max_log2 - b->p.dt_min_log2;
    const bool split = b->p.precision == NB_SPLIT;
    // jobs in the batch and not failed
    int nj = 0;
    for (int k = 0; k < b->p.max_jobs; ++k)
        if (b->alive[k])
            b->h_jobs[nj++] = k;
    int64_t inter = 0;
    if (nj > 0) {
        B_HIP(b, hipMemcpyAsync(b->d_jobs, b->h_jobs, 4 * (size_t)nj, hipMemcpyHostToDevice, b->st));
        hipLaunchKernelGGL(nb::k_bact, dim3(nj), dim3(nb::kBS), 0, b->st, b->P, (const int32_t *)b->d_jobs, L);
        B_HIP(b, hipGetLastError());
        nb_status s = b_fetch_jobs(b);
        if (s) return s;
        std::vector<int> group;
        for (int k = 0; k < nj; ++k) {
            const int job = b->h_jobs[k];
            if (b->h_err[job]) {
                b->h_nact[job] = 0;  // a failed job is not stepped again
                continue;
            }
            if (b->h_nact[job] > 0) {
                group.push_back(job);
                inter += b->h_nact[job] * b->n[job];
            }
        }
        if (!group.empty()) {
            // failed jobs must not be predicted either
            B_HIP(b, hipMemcpyAsync(b->P.j_nact, b->h_nact, 8 * (size_t)b->p.max_jobs,
                                    hipMemcpyHostToDevice, b->st));
            hipLaunchKernelGGL(nb::k_bpredict, dim3(nb::nblk(b->cap, 256)), dim3(256), 0, b->st, b->P, b->cap,
                               ldexp(1.0, b->p.dt_min_log2), (int)split);
            B_HIP(b, hipGetLastError());
            if ((s = b_evaluate(b, group))) return s;
            if ((s = b_correct_levels(b, group, 0))) return s;
            B_HIP(b, hipMemcpyAsync(b->h_err, b->P.j_err, 4 * (size_t)b->p.max_jobs, hipMemcpyDeviceToHost,
                                    b->st));
            B_HIP(b, hipStreamSynchronize(b->st));
        }
    }
    for (int k = 0; k < b->p.max_jobs; ++k) {
        const bool live = b->alive[k];
        if (h_n_act) h_n_act[k] = live ? b->h_nact[k] : 0;
        if (h_tick_next) h_tick_next[k] = live ? b->h_tnext[k] : 0;
        if (h_job_err) h_job_err[k] = live ? b->h_err[k] : 0;
    }
    if (h_interactions)
        *h_interactions = inter;
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
