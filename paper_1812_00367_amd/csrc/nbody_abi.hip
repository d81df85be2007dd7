// nbody_abi.hip -- host side of the C ABI declared in include/nbody.h: argument
// checks, workspace layout, call ordering, error latching and kernel dispatch.
// No device memory is allocated here; every array lives in the caller's workspace.
#include "nbody.h"
#include "nb_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

using nb::Arrays;
using nb::Status;

struct nb_ctx {
    nb_params p;
    hipStream_t st;
    int device;
    Arrays A;
    size_t bytes;
    Status *h_status;  // pinned host copy of the device status block
    char msg[512];
    bool have_state;
    bool synced;       // every body at sync_tick (nb_set_state without tick array)
    int64_t sync_tick;
    bool predicted;    // j-records hold a prediction that no correction has invalidated
    int64_t pred_tick; // the time of that prediction
    const int32_t *eval_idx;
    int64_t eval_n;
    bool eval_valid;   // an evaluation is waiting for its correction
    int32_t cfg[4];    // forced launch shape (all zero: use the table)
    nb::EvalRow rows[nb::kMaxEvalRows];  // launch table (nrows == 0: built-in)
    int nrows;
};

namespace {

constexpr int64_t kMaxN = (int64_t)1 << 30;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Full evaluations (every body active) of systems of at least kSymMinN bodies take
// the pairwise-symmetric kernel when its partial sums fit the partial buffer; the
// default buffer holds them up to kSymDefaultMaxN bodies.
constexpr int64_t kSymMinN = 8192;
constexpr int64_t kSymDefaultMaxN = 65536;

// Partial-sum slots (10 doubles each) of the symmetric evaluation: one for its unit
// counter, then its row and column buffers.
int64_t sym_slots(int64_t n)
{
    const nb::SymPlan S = nb::plan_sym(n, nb::kSymGroups);
    return 1 + (S.row_slots + S.col_slots + 9) / 10;
}

int64_t partial_slots_of(const nb_params *p)
{
    if (p->partial_slots > 0)
        return p->partial_slots;
    const int64_t a = 4 * p->n, b = (int64_t)1 << 20;
    int64_t s = a > b ? a : b;
    if (p->precision == NB_FP64 && p->n >= kSymMinN && p->n <= kSymDefaultMaxN) {
        const int64_t need = sym_slots(p->n);
        s = need > s ? need : s;
    }
    return s;
}

// Carve the workspace (base may be null to only measure). Returns the total size.
size_t layout(const nb_params *p, Arrays *A, char *base)
{
    const size_t n = (size_t)p->n;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = align256(off);
        void *r = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return r;
    };
    const bool split = p->precision == NB_SPLIT;
    A->m = (double *)take(8 * n);
    A->x = (double *)take(24 * n);
    A->v = (double *)take(24 * n);
    A->a = (double *)take(24 * n);
    A->j = (double *)take(24 * n);
    A->s = (double *)take(24 * n);
    A->c = (double *)take(24 * n);
    A->a4n = (double *)take(8 * n);
    A->a5n = (double *)take(8 * n);
    A->phi = (double *)take(8 * n);
    A->tick = (int64_t *)take(8 * n);
    A->level = (int32_t *)take(4 * n);
    A->jrec = (double *)take(8 * nb::kRecD * n);
    A->jrec32 = split ? (float *)take(4 * nb::kRecF * n) : nullptr;
    A->evalbuf = (double *)take(80 * n);
    A->part = (double *)take(80 * (size_t)partial_slots_of(p));
    A->act_idx = (int32_t *)take(4 * n);
    A->act_bmin = (int64_t *)take(8 * (size_t)nb::act_blocks(p->n));
    A->act_bcnt = (int32_t *)take(4 * (size_t)nb::act_blocks(p->n));
    A->en_bsum = (double *)take(16 * (size_t)nb::en_blocks(p->n));
    A->status = (Status *)take(sizeof(Status));
    A->jrecj = (double *)take(32 * n);
    A->crk = (p->flags & NB_FLAG_START_CRACKLE) ? (double *)take(104 * n) : nullptr;
    A->ectr = (unsigned *)take(4 * (size_t)nb::kMaxGroups);
    return align256(off);
}

nb_status fail(nb_ctx *c, nb_status s, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->msg, sizeof c->msg, fmt, ap);
        va_end(ap);
    }
    return s;
}

const char *check_params(const nb_params *p)
{
    if (!p) return "params is NULL";
    if (p->n < 1 || p->n > kMaxN) return "n must be in [1, 2^30]";
    if (!(p->eps >= 0.0) || !isfinite(p->eps)) return "eps must be finite and >= 0";
    if (!(p->eta > 0.0) || !isfinite(p->eta)) return "eta must be finite and > 0";
    if (!(p->eta_init > 0.0) || !isfinite(p->eta_init)) return "eta_init must be finite and > 0";
    if (p->dt_max_log2 > 100 || p->dt_min_log2 < -200) return "dt_max_log2 <= 100 and dt_min_log2 >= -200";
    const int L = p->dt_max_log2 - p->dt_min_log2;
    if (L < 0 || L > 62) return "need 0 <= dt_max_log2 - dt_min_log2 <= 62";
    if (p->precision != NB_FP64 && p->precision != NB_SPLIT) return "precision must be NB_FP64 or NB_SPLIT";
    if (p->flags & ~NB_FLAG_START_CRACKLE) return "unknown flags";
    if (p->partial_slots < 0) return "partial_slots must be >= 0";
    return nullptr;
}

#define NB_HIP(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), NB_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

#define NB_CTX(ctx)                                                                        \
    do {                                                                                   \
        if (!(ctx)) return NB_ERR_ARG;                                                     \
        (ctx)->msg[0] = 0;                                                                 \
    } while (0)

// Wait for the stream, fetch the status block and turn latched device errors into
// a status (clearing them).
nb_status sync_status(nb_ctx *c)
{
    NB_HIP(c, hipMemcpyAsync(c->h_status, c->A.status, sizeof(Status), hipMemcpyDeviceToHost, c->st));
    NB_HIP(c, hipStreamSynchronize(c->st));
    const int32_t *e = c->h_status->err;
    if (e[nb::kErrIndex] || e[nb::kErrLevel] || e[nb::kErrNumeric] || e[nb::kErrDtMin]) {
        nb_status s;
        if (e[nb::kErrIndex])
            s = fail(c, NB_ERR_ARG, "an index list entry is outside [0, n), or the list given to nb_correct is "
                                    "not strictly ascending");
        else if (e[nb::kErrLevel])
            s = fail(c, NB_ERR_ARG, "a body's time or level is inconsistent with the call "
                                    "(level outside [0, L], or a body ahead of the target time)");
        else if (e[nb::kErrNumeric])
            s = fail(c, NB_ERR_NUMERIC, "a non-finite value (start-up evaluation or corrector)");
        else
            s = fail(c, NB_ERR_NUMERIC, "a body needs a step below 2^dt_min_log2");
        NB_HIP(c, nb::launch_fill_i32(c->A.status->err, 0, nb::kErrWords, c->st));
        NB_HIP(c, hipStreamSynchronize(c->st));
        return s;
    }
    return NB_OK;
}

nb_status check_idx(nb_ctx *c, const int32_t *idx, int64_t n_act)
{
    if (n_act < 0 || n_act > c->p.n)
        return fail(c, NB_ERR_ARG, "n_act = %lld outside [0, n]", (long long)n_act);
    if (n_act > 0 && !idx)
        return fail(c, NB_ERR_ARG, "index list is NULL");
    return NB_OK;
}

nb_status do_predict(nb_ctx *c, int64_t tick)
{
    NB_HIP(c, nb::launch_predict(c->A, c->p.n, tick, c->p.dt_min_log2, c->p.precision == NB_SPLIT, c->st));
    c->predicted = true;
    c->pred_tick = tick;
    return NB_OK;
}

// Whether an evaluation of n_act bodies takes the pairwise-symmetric kernel: FP64,
// every body active, no forced launch shape, and room for its partial sums.
bool use_sym(const nb_ctx *c, int64_t n_act)
{
    if (c->p.precision != NB_FP64 || c->cfg[0] || n_act != c->p.n || c->p.n < kSymMinN)
        return false;
    return sym_slots(c->p.n) <= partial_slots_of(&c->p);
}

nb::EvalPlan make_plan(const nb_ctx *c, int64_t n_act)
{
    if (c->cfg[0])
        return nb::plan_eval_fixed(c->p.n, n_act, c->cfg[0], c->cfg[1], c->cfg[2], c->cfg[3]);
    return nb::plan_eval(c->p.n, n_act, partial_slots_of(&c->p), c->p.precision == NB_SPLIT,
                         c->rows, c->nrows);
}

nb_status do_evaluate(nb_ctx *c, const int32_t *idx, int64_t n_act, double *out)
{
    if (n_act > 0 && use_sym(c, n_act)) {
        const nb::SymPlan S = nb::plan_sym(c->p.n, nb::kSymGroups);
        unsigned *claim = reinterpret_cast<unsigned *>(c->A.part);
        double *rowbuf = c->A.part + 10, *colbuf = rowbuf + S.row_slots;
        NB_HIP(c, nb::launch_eval_sym(c->A, S, c->p.n, idx, n_act, c->p.eps, rowbuf, colbuf, claim,
                                      c->A.evalbuf, out, c->st));
    } else if (n_act > 0) {
        const nb::EvalPlan P = make_plan(c, n_act);
        if (P.splits > 1 && (int64_t)P.splits * n_act > partial_slots_of(&c->p))
            return fail(c, NB_ERR_SPACE, "partial-sum buffer too small");
        NB_HIP(c, nb::launch_eval(c->A, P, c->p.n, idx, n_act, c->p.eps, c->p.precision == NB_SPLIT, out, c->st));
    }
    c->eval_idx = idx;
    c->eval_n = n_act;
    c->eval_valid = true;
    return NB_OK;
}

}  // namespace

namespace nb {

// Launch shapes. The chip has 256 CUs x 4 SIMDs: a launch wants a few waves per
// SIMD, while the partial-sum traffic (S x n_act x 80 bytes) stays small against
// the O(n_act n) arithmetic. The built-in tables were picked by
// paper_1812_00367_amd/tune.py on an MI355X (N = 65536, both precisions; FP64 from a
// sweep of 1 ... 32768 active bodies over the broadcast, small-set and group
// kernels) and checked by timings of the candidates at 1, 64, 1024 and 8192 active
// bodies.
static const EvalRow kDefaultF64[] = {
    {1, -1, 1, 0, 256},     {2, -2, 1, 0, 512},      {5, -4, 4, 0, 1024},
    {11, -8, 4, 256, 1024}, {22, -16, 8, 256, 2048}, {45, -32, 8, 256, 2048},
    {90, -32, 8, 256, 4096}, {181, -32, 4, 256, 4096}, {362, -64, 8, 256, 4096},
    {724, -64, 8, 256, 8192}, {1448, -64, 4, 256, 8192}, {5792, -128, 4, 256, 8192},
    {11585, -128, 4, 256, 4096},
    {23170, 2, 1, 64, 8192}, {1 << 30, -128, 4, 256, 16384},
};
static const EvalRow kDefaultSplit[] = {
    {128, 1, 1, 64, 1024},
    {2048, 1, 2, 128, 2048},
    {8192, 1, 4, 256, 8192},
    {1 << 30, 1, 4, 256, 16384},
};

bool eval_shape_supported(int ipl, int waves, int tile, bool split)
{
    if (ipl < 0) {
        const int pmax = -ipl;
        if (split)
            return false;
        if (waves > 1)
            return group_shape_ok(pmax, waves, tile);
        return pmax <= 64 && (pmax & (pmax - 1)) == 0 && waves == 1 &&
               (tile == 64 || tile == 0);
    }
    if (ipl != 1 && ipl != 2)
        return false;
    return (waves == 1 && (tile == 64 || tile == 128 || tile == 256)) ||
           (waves == 2 && (tile == 128 || tile == 256)) || (waves == 4 && tile == 256);
}

// The j-split of n bodies into about S ranges of whole `unit`-record blocks.
static void split_range(int64_t n, int64_t S, int unit, EvalPlan &P)
{
    const int64_t max_units = (n + unit - 1) / unit;
    if (S > max_units) S = max_units;
    if (S < 1) S = 1;
    int64_t per = (n + S - 1) / S;
    per = (per + unit - 1) / unit * unit;
    P.jchunk = (int)per;
    P.splits = (int)((n + per - 1) / per);
}

// Group kernel: G = the power of two >= n_act, at most Pmax (and, with LDS tiles, at
// least 64 waves / 256 so that the lane slots divide a tile); W = 64 / G lanes per
// body (G = 128: two bodies per lane).
static void plan_group(int64_t n, int64_t n_act, int pmax, int waves, int tile, int64_t S,
                       EvalPlan &P)
{
    int G = 1;
    while (G < n_act && G < pmax)
        G <<= 1;
    if (tile > 0)
        while (waves * (64 / (G < 64 ? G : 64)) > kGroupTile)
            G <<= 1;
    P.ipl = -G;
    P.lw = 0;
    while ((64 >> P.lw) > G)
        ++P.lw;
    P.iblocks = (int)((n_act + G - 1) / G);
    split_range(n, S, tile > 0 ? kGroupTile : 64, P);
    const int64_t cnt = n_act < G ? n_act : G;
    P.fused = P.splits > 1 && P.iblocks <= kMaxGroups &&
              (int64_t)P.splits * cnt * 10 <= (int64_t)kTailPerThread * 64 * waves;
}

EvalPlan plan_eval_fixed(int64_t n, int64_t n_act, int ipl, int waves, int tile, int64_t S)
{
    EvalPlan P{};
    P.waves = waves;
    P.tile = tile;
    if (ipl < 0 && waves > 1) {
        plan_group(n, n_act, -ipl, waves, tile, S, P);
        return P;
    }
    if (ipl < 0) {
        // small-set kernel: P active bodies per wave, 64 / P lanes each
        int pw = 1;
        while (pw < n_act && pw < -ipl)
            pw <<= 1;
        P.ipl = -pw;
        P.lw = 0;
        while ((64 >> P.lw) > pw)
            ++P.lw;
        P.iblocks = (int)((n_act + pw - 1) / pw);
        split_range(n, S, kLaneTile, P);
        return P;
    }
    P.ipl = ipl;
    P.lw = -1;
    const int64_t per_block = (int64_t)ipl * 64 * waves;
    P.iblocks = (int)((n_act + per_block - 1) / per_block);
    split_range(n, S, tile, P);
    return P;
}

EvalPlan plan_eval(int64_t n, int64_t n_act, int64_t partial_slots, bool split,
                   const EvalRow *rows, int nrows)
{
    if (nrows <= 0) {
        rows = split ? kDefaultSplit : kDefaultF64;
        nrows = (int)((split ? sizeof kDefaultSplit : sizeof kDefaultF64) / sizeof(EvalRow));
    }
    const EvalRow *r = &rows[nrows - 1];
    for (int k = 0; k < nrows; ++k)
        if (n_act <= rows[k].n_act_max) {
            r = &rows[k];
            break;
        }
    // waves along the active bodies, then S ~ target / that
    int64_t waves_i;
    if (r->ipl < 0) {
        int64_t pw = 1;
        while (pw < n_act && pw < -r->ipl)
            pw <<= 1;
        waves_i = (n_act + pw - 1) / pw * r->waves;  // group kernel: its waves share a group
    } else {
        const int64_t per_block = (int64_t)r->ipl * 64 * r->waves;
        waves_i = (n_act + per_block - 1) / per_block * r->waves;
    }
    int64_t S = (r->target_waves + waves_i - 1) / waves_i;
    const int64_t cap = partial_slots / (n_act > 0 ? n_act : 1);
    if (S > cap) S = cap;
    return plan_eval_fixed(n, n_act, r->ipl, r->waves, r->tile, S);
}

}  // namespace nb

namespace {

// Device memory of nb_evaluate_static: one file-scope array per device (each GPU the
// library runs on holds its own copy until the process ends). Host code never uses
// the array's name as an address: the device address comes from hipGetSymbolAddress,
// once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[NB_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Layout of the array: the status block, the group kernel's counters (zeroed once per
// device, then left at zero by every launch), the j-records, the partial sums.
constexpr size_t kScratchCtrOff = (sizeof(Status) + 255) / 256 * 256;
constexpr size_t kScratchRecOff = kScratchCtrOff + 4 * (size_t)nb::kMaxGroups;

// The device address of `scratch` on the current device (nullptr on failure). The
// first call on a device also enqueues the zeroing of the counters on st.
void *scratch_on_current_device(hipError_t *err, hipStream_t st)
{
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess)
        return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess || !ptr)
            return nullptr;
        *err = nb::launch_fill_i32((int32_t *)((char *)ptr + kScratchCtrOff), 0, nb::kMaxGroups, st);
        if (*err != hipSuccess)
            return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

nb_status nb_workspace_bytes(const nb_params *p, size_t *h_bytes)
{
    if (!h_bytes || check_params(p))
        return NB_ERR_ARG;
    Arrays A{};
    *h_bytes = layout(p, &A, nullptr);
    return NB_OK;
}

nb_status nb_create(const nb_params *p, void *d_workspace, size_t bytes, nb_ctx **out)
{
    if (!out)
        return NB_ERR_ARG;
    *out = nullptr;
    if (check_params(p) || !d_workspace || ((uintptr_t)d_workspace & 255))
        return NB_ERR_ARG;
    Arrays A{};
    const size_t need = layout(p, &A, nullptr);
    if (bytes < need)
        return NB_ERR_SPACE;
    nb_ctx *c = new (std::nothrow) nb_ctx();
    if (!c)
        return NB_ERR_SPACE;
    c->p = *p;
    c->st = (hipStream_t)p->stream;
    c->bytes = bytes;
    layout(p, &c->A, (char *)d_workspace);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipHostMalloc((void **)&c->h_status, sizeof(Status), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return NB_ERR_DEVICE;
    }
    memset(c->h_status, 0, sizeof(Status));
    // zero the whole state and the status block
    const size_t n = (size_t)p->n;
    hipError_t e = hipSuccess;
    for (double *q : {c->A.m, c->A.a4n, c->A.a5n, c->A.phi})
        if (e == hipSuccess) e = nb::launch_fill_f64(q, 0.0, n, c->st);
    for (double *q : {c->A.x, c->A.v, c->A.a, c->A.j, c->A.s, c->A.c})
        if (e == hipSuccess) e = nb::launch_fill_f64(q, 0.0, 3 * n, c->st);
    if (e == hipSuccess) e = nb::launch_fill_i32((int32_t *)c->A.ectr, 0, nb::kMaxGroups, c->st);
    if (e == hipSuccess) e = nb::launch_fill_i64(c->A.tick, 0, n, c->st);
    if (e == hipSuccess) e = nb::launch_fill_i32(c->A.level, 0, n, c->st);
    if (e == hipSuccess) e = nb::launch_fill_i32((int32_t *)c->A.status, 0, sizeof(Status) / 4, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) {
        (void)hipHostFree(c->h_status);
        delete c;
        return NB_ERR_DEVICE;
    }
    *out = c;
    return NB_OK;
}

void nb_destroy(nb_ctx *c)
{
    if (!c)
        return;
    (void)hipStreamSynchronize(c->st);
    (void)hipHostFree(c->h_status);
    delete c;
}

const char *nb_last_error(const nb_ctx *c) { return c ? c->msg : "null context"; }

nb_status nb_set_state(nb_ctx *c, const nb_state *src, int64_t tick0)
{
    NB_CTX(c);
    if (!src || !src->m || !src->x || !src->v)
        return fail(c, NB_ERR_ARG, "m, x and v are required");
    const size_t n = (size_t)c->p.n;
    const Arrays &A = c->A;
    auto cp = [&](void *dst, const void *s, size_t bytes) {
        return hipMemcpyAsync(dst, s, bytes, hipMemcpyDeviceToDevice, c->st);
    };
    NB_HIP(c, cp(A.m, src->m, 8 * n));
    NB_HIP(c, cp(A.x, src->x, 24 * n));
    NB_HIP(c, cp(A.v, src->v, 24 * n));
    struct V3 { double *d; const double *s; } v3[] = {{A.a, src->a}, {A.j, src->j}, {A.s, src->s}, {A.c, src->c}};
    for (auto &f : v3) {
        if (f.s) NB_HIP(c, cp(f.d, f.s, 24 * n));
        else NB_HIP(c, nb::launch_fill_f64(f.d, 0.0, 3 * n, c->st));
    }
    struct V1 { double *d; const double *s; } v1[] = {{A.a4n, src->a4n}, {A.a5n, src->a5n}};
    for (auto &f : v1) {
        if (f.s) NB_HIP(c, cp(f.d, f.s, 8 * n));
        else NB_HIP(c, nb::launch_fill_f64(f.d, 0.0, n, c->st));
    }
    NB_HIP(c, nb::launch_fill_f64(A.phi, 0.0, n, c->st));
    if (src->tick) {
        NB_HIP(c, cp(A.tick, src->tick, 8 * n));
        c->synced = false;
    } else {
        NB_HIP(c, nb::launch_fill_i64(A.tick, tick0, n, c->st));
        c->synced = true;
        c->sync_tick = tick0;
    }
    if (src->level) NB_HIP(c, cp(A.level, src->level, 4 * n));
    else NB_HIP(c, nb::launch_fill_i32(A.level, 0, n, c->st));
    c->have_state = true;
    c->predicted = false;
    c->eval_valid = false;
    return NB_OK;
}

nb_status nb_set_times(nb_ctx *c, const int64_t *d_tick, const int32_t *d_level)
{
    NB_CTX(c);
    if (!d_tick || !d_level)
        return fail(c, NB_ERR_ARG, "tick and level are required");
    if (!c->have_state)
        return fail(c, NB_ERR_STATE, "no state loaded");
    const size_t n = (size_t)c->p.n;
    NB_HIP(c, hipMemcpyAsync(c->A.tick, d_tick, 8 * n, hipMemcpyDeviceToDevice, c->st));
    NB_HIP(c, hipMemcpyAsync(c->A.level, d_level, 4 * n, hipMemcpyDeviceToDevice, c->st));
    c->synced = false;
    c->predicted = false;
    c->eval_valid = false;
    return NB_OK;
}

nb_status nb_get_state(nb_ctx *c, const nb_state *dst)
{
    NB_CTX(c);
    if (!dst)
        return fail(c, NB_ERR_ARG, "dst is NULL");
    const size_t n = (size_t)c->p.n;
    const Arrays &A = c->A;
    auto cp = [&](void *d, const void *s, size_t bytes) {
        return d ? hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, c->st) : hipSuccess;
    };
    NB_HIP(c, cp(dst->m, A.m, 8 * n));
    NB_HIP(c, cp(dst->x, A.x, 24 * n));
    NB_HIP(c, cp(dst->v, A.v, 24 * n));
    NB_HIP(c, cp(dst->a, A.a, 24 * n));
    NB_HIP(c, cp(dst->j, A.j, 24 * n));
    NB_HIP(c, cp(dst->s, A.s, 24 * n));
    NB_HIP(c, cp(dst->c, A.c, 24 * n));
    NB_HIP(c, cp(dst->a4n, A.a4n, 8 * n));
    NB_HIP(c, cp(dst->a5n, A.a5n, 8 * n));
    NB_HIP(c, cp(dst->phi, A.phi, 8 * n));
    NB_HIP(c, cp(dst->tick, A.tick, 8 * n));
    NB_HIP(c, cp(dst->level, A.level, 4 * n));
    return sync_status(c);
}

nb_status nb_start(nb_ctx *c)
{
    NB_CTX(c);
    if (!c->have_state || !c->synced)
        return fail(c, NB_ERR_STATE, "nb_start needs a synchronised state from nb_set_state");
    const int64_t n = c->p.n;
    const bool split = c->p.precision == NB_SPLIT;
    int32_t *all = c->A.act_idx;  // idx = 0..n-1 in the workspace's active list
    NB_HIP(c, nb::launch_iota(all, n, c->st));
    nb_status s = do_predict(c, c->sync_tick);
    if (s) return s;
    if ((s = do_evaluate(c, all, n, nullptr))) return s;
    NB_HIP(c, nb::launch_copy_acc_to_jrec(c->A, n, split, c->st));
    if ((s = do_evaluate(c, all, n, nullptr))) return s;
    NB_HIP(c, nb::launch_start_store(c->A, n, c->st));
    if (c->p.flags & NB_FLAG_START_CRACKLE) {
        // third pass: crackle from the same predicted records plus the jerks just found
        NB_HIP(c, nb::launch_eval_crackle(c->A, n, all, n, c->p.eps, partial_slots_of(&c->p), c->sync_tick,
                                          c->p.dt_min_log2, c->A.crk, c->st));
        NB_HIP(c, nb::launch_store_crackle(c->A, n, c->A.crk, c->st));
    }
    NB_HIP(c, nb::launch_timesteps(c->A, n, all, n, 1, c->p.eta, c->p.eta_init, c->p.dt_max_log2,
                                   c->p.dt_min_log2, c->st));
    c->eval_valid = false;
    c->synced = false;
    return NB_OK;
}

nb_status nb_active(nb_ctx *c, int32_t *d_idx_out, int64_t *h_n_act, int64_t *h_tick_next)
{
    NB_CTX(c);
    if (!d_idx_out || !h_n_act || !h_tick_next)
        return fail(c, NB_ERR_ARG, "NULL output");
    NB_HIP(c, nb::launch_active(c->A, c->p.n, c->p.dt_max_log2 - c->p.dt_min_log2, d_idx_out, c->st));
    nb_status s = sync_status(c);
    if (s)
        return s;
    *h_n_act = c->h_status->n_act;
    *h_tick_next = c->h_status->tick_next;
    return NB_OK;
}

nb_status nb_predict(nb_ctx *c, int64_t tick)
{
    NB_CTX(c);
    if (!c->have_state)
        return fail(c, NB_ERR_STATE, "no state loaded");
    return do_predict(c, tick);
}

nb_status nb_get_predicted(nb_ctx *c, double *d_xp, double *d_vp, double *d_ap)
{
    NB_CTX(c);
    if (!c->predicted)
        return fail(c, NB_ERR_STATE, "no current prediction");
    NB_HIP(c, nb::launch_get_predicted(c->A, c->p.n, d_xp, d_vp, d_ap, c->st));
    return NB_OK;
}

nb_status nb_evaluate(nb_ctx *c, const int32_t *d_idx, int64_t n_act, double *d_out)
{
    NB_CTX(c);
    nb_status s = check_idx(c, d_idx, n_act);
    if (s)
        return s;
    if (!c->predicted)
        return fail(c, NB_ERR_STATE, "nb_evaluate needs a prediction (nb_predict) first");
    return do_evaluate(c, d_idx, n_act, d_out);
}

nb_status nb_evaluate_crackle(nb_ctx *c, const int32_t *d_idx, int64_t n_act, double *d_out)
{
    NB_CTX(c);
    nb_status s = check_idx(c, d_idx, n_act);
    if (s)
        return s;
    if (n_act > 0 && !d_out)
        return fail(c, NB_ERR_ARG, "d_out is NULL");
    if (!c->predicted)
        return fail(c, NB_ERR_STATE, "nb_evaluate_crackle needs a prediction (nb_predict) first");
    if ((int64_t)13 * n_act > 10 * partial_slots_of(&c->p))
        return fail(c, NB_ERR_SPACE, "partial-sum buffer too small for %lld active bodies", (long long)n_act);
    NB_HIP(c, nb::launch_eval_crackle(c->A, c->p.n, d_idx, n_act, c->p.eps, partial_slots_of(&c->p),
                                      c->pred_tick, c->p.dt_min_log2, d_out, c->st));
    return NB_OK;
}

nb_status nb_evaluate_static(int64_t n, const double *d_m, const double *d_xp, const double *d_vp,
                             const double *d_ap, double eps, const int32_t *d_idx, int64_t n_act,
                             double *d_out, void *stream)
{
    if (n < 1 || n > kMaxN || n_act < 0 || n_act > n || !(eps >= 0.0) || !isfinite(eps))
        return NB_ERR_ARG;
    if (n_act == 0)
        return NB_OK;
    if (!d_m || !d_xp || !d_vp || !d_ap || !d_idx || !d_out)
        return NB_ERR_ARG;
    // the launch shape nb_evaluate uses for a context of n bodies with the default
    // partial-sum capacity and the built-in table (the one-sided kernels only), so
    // both give the same bits whenever nb_evaluate takes those kernels
    nb_params dp{};
    dp.n = n;
    dp.precision = NB_FP64;
    const nb::EvalPlan P = nb::plan_eval(n, n_act, partial_slots_of(&dp), false, nullptr, 0);
    const size_t rec_bytes = align256(80 * (size_t)n);
    const size_t part_bytes = P.splits > 1 ? align256(80 * (size_t)P.splits * (size_t)n_act) : 0;
    const size_t need = kScratchRecOff + rec_bytes + part_bytes;
    if (need > NB_STATIC_SCRATCH_BYTES)
        return NB_ERR_SPACE;
    hipError_t e = hipSuccess;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)scratch_on_current_device(&e, st);
    if (!base)
        return NB_ERR_DEVICE;
    Arrays A{};
    A.status = (Status *)base;
    A.ectr = (unsigned *)(base + kScratchCtrOff);
    A.jrec = (double *)(base + kScratchRecOff);
    A.part = P.splits > 1 ? (double *)((char *)A.jrec + rec_bytes) : nullptr;
    A.evalbuf = d_out;  // the kernels write (or reduce into) the caller's output
    // the scratch keeps the last call's contents: clear the error words (a fill
    // kernel, which graph capture records as a kernel node)
    if ((e = nb::launch_fill_i32(A.status->err, 0, nb::kErrWords, st)) != hipSuccess)
        return NB_ERR_DEVICE;
    if ((e = nb::launch_pack_records(d_m, d_xp, d_vp, d_ap, n, A.jrec, st)) != hipSuccess)
        return NB_ERR_DEVICE;
    if ((e = nb::launch_eval(A, P, n, d_idx, n_act, eps, false, nullptr, st)) != hipSuccess)
        return NB_ERR_DEVICE;
    if ((e = nb::launch_poison_on_index_error(A.status, d_out, 10 * n_act, st)) != hipSuccess)
        return NB_ERR_DEVICE;
    return NB_OK;
}

nb_status nb_set_evaluation(nb_ctx *c, const int32_t *d_idx, int64_t n_act, const double *d_in)
{
    NB_CTX(c);
    nb_status s = check_idx(c, d_idx, n_act);
    if (s)
        return s;
    if (n_act > 0 && !d_in)
        return fail(c, NB_ERR_ARG, "d_in is NULL");
    if (n_act > 0)
        NB_HIP(c, hipMemcpyAsync(c->A.evalbuf, d_in, sizeof(double) * 10 * (size_t)n_act,
                                 hipMemcpyDeviceToDevice, c->st));
    c->eval_idx = d_idx;
    c->eval_n = n_act;
    c->eval_valid = true;
    return NB_OK;
}

nb_status nb_eval_config(nb_ctx *c, const int32_t *h_cfg, int64_t n_act, int32_t *h_shape_out)
{
    NB_CTX(c);
    int32_t cfg[4] = {0, 0, 0, 0};
    if (h_cfg)
        memcpy(cfg, h_cfg, sizeof cfg);
    const bool zero = !cfg[0] && !cfg[1] && !cfg[2] && !cfg[3];
    if (!zero) {
        const bool ok = cfg[3] >= 1 &&
                        nb::eval_shape_supported(cfg[0], cfg[1], cfg[2], c->p.precision == NB_SPLIT);
        if (!ok)
            return fail(c, NB_ERR_ARG, "unsupported launch shape {%d,%d,%d,%d}", cfg[0], cfg[1],
                        cfg[2], cfg[3]);
    }
    memcpy(c->cfg, cfg, sizeof cfg);
    if (h_shape_out) {
        if (n_act < 1 || n_act > c->p.n)
            return fail(c, NB_ERR_ARG, "n_act outside [1, n]");
        if (use_sym(c, n_act)) {
            const nb::SymPlan S = nb::plan_sym(c->p.n, nb::kSymGroups);
            h_shape_out[0] = 0;
            h_shape_out[1] = nb::kSymWaves;
            h_shape_out[2] = 64;
            h_shape_out[3] = S.B / S.parts;
            h_shape_out[4] = (int32_t)S.items;
            h_shape_out[5] = S.G;
            h_shape_out[6] = 0;
            return NB_OK;
        }
        const nb::EvalPlan P = make_plan(c, n_act);
        h_shape_out[0] = P.ipl;
        h_shape_out[1] = P.waves;
        h_shape_out[2] = P.tile;
        h_shape_out[3] = P.jchunk;
        h_shape_out[4] = P.splits;
        h_shape_out[5] = P.iblocks;
        h_shape_out[6] = P.fused;
    }
    return NB_OK;
}

nb_status nb_eval_table(nb_ctx *c, const int32_t *h_rows, int32_t nrows)
{
    NB_CTX(c);
    if (nrows < 0 || nrows > nb::kMaxEvalRows || (nrows > 0 && !h_rows))
        return fail(c, NB_ERR_ARG, "nrows must be in [0, %d]", nb::kMaxEvalRows);
    for (int k = 0; k < nrows; ++k) {
        const int32_t *r = h_rows + 5 * k;
        if (r[0] < 1 || (k > 0 && r[0] <= h_rows[5 * (k - 1)]) || r[4] < 1 ||
            !nb::eval_shape_supported(r[1], r[2], r[3], c->p.precision == NB_SPLIT))
            return fail(c, NB_ERR_ARG, "bad table row %d {%d,%d,%d,%d,%d}", k, r[0], r[1], r[2],
                        r[3], r[4]);
    }
    for (int k = 0; k < nrows; ++k) {
        const int32_t *r = h_rows + 5 * k;
        c->rows[k] = nb::EvalRow{r[0], r[1], r[2], r[3], r[4]};
    }
    c->nrows = nrows;
    return NB_OK;
}

nb_status nb_correct(nb_ctx *c, const int32_t *d_idx, int64_t n_act, int64_t tick)
{
    NB_CTX(c);
    nb_status s = check_idx(c, d_idx, n_act);
    if (s)
        return s;
    if (!c->eval_valid || d_idx != c->eval_idx || n_act != c->eval_n)
        return fail(c, NB_ERR_STATE, "nb_correct must follow nb_evaluate with the same index list");
    NB_HIP(c, nb::launch_correct(c->A, c->p.n, d_idx, n_act, tick, c->p.dt_min_log2, c->st));
    c->eval_valid = false;
    c->predicted = false;
    return NB_OK;
}

nb_status nb_timesteps(nb_ctx *c, const int32_t *d_idx, int64_t n_act, int init)
{
    NB_CTX(c);
    nb_status s = check_idx(c, d_idx, n_act);
    if (s)
        return s;
    if (!c->have_state)
        return fail(c, NB_ERR_STATE, "no state loaded");
    NB_HIP(c, nb::launch_timesteps(c->A, c->p.n, d_idx, n_act, init ? 1 : 0, c->p.eta, c->p.eta_init,
                                   c->p.dt_max_log2, c->p.dt_min_log2, c->st));
    return NB_OK;
}

nb_status nb_step(nb_ctx *c, int64_t tick_limit, int64_t *h_n_act, int64_t *h_tick_next)
{
    NB_CTX(c);
    if (!h_n_act || !h_tick_next)
        return fail(c, NB_ERR_ARG, "NULL output");
    if (!c->have_state)
        return fail(c, NB_ERR_STATE, "no state loaded");
    int64_t na = 0, tn = 0;
    nb_status s = nb_active(c, c->A.act_idx, &na, &tn);
    if (s)
        return s;
    *h_tick_next = tn;
    if (tick_limit >= 0 && tn > tick_limit) {
        *h_n_act = 0;
        return NB_OK;
    }
    if ((s = do_predict(c, tn))) return s;
    if ((s = do_evaluate(c, c->A.act_idx, na, nullptr))) return s;
    NB_HIP(c, nb::launch_correct(c->A, c->p.n, c->A.act_idx, na, tn, c->p.dt_min_log2, c->st));
    NB_HIP(c, nb::launch_timesteps(c->A, c->p.n, c->A.act_idx, na, 0, c->p.eta, c->p.eta_init,
                                   c->p.dt_max_log2, c->p.dt_min_log2, c->st));
    c->eval_valid = false;
    c->predicted = false;
    *h_n_act = na;
    return NB_OK;
}

nb_status nb_energy(nb_ctx *c, int64_t tick, double *h_ekin, double *h_epot)
{
    NB_CTX(c);
    if (!h_ekin || !h_epot)
        return fail(c, NB_ERR_ARG, "NULL output");
    if (!c->have_state)
        return fail(c, NB_ERR_STATE, "no state loaded");
    nb_status s = do_predict(c, tick);
    if (s)
        return s;
    NB_HIP(c, nb::launch_energy(c->A, c->p.n, c->p.eps, partial_slots_of(&c->p), c->st));
    if ((s = sync_status(c)))
        return s;
    *h_ekin = c->h_status->ekin;
    *h_epot = c->h_status->epot;
    return NB_OK;
}

}  // extern "C"
