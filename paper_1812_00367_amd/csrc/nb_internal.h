// nb_internal.h -- private interface between the host ABI (nbody_abi.hip) and the
// gfx950 kernels (nbody_kernels.hip). Not installed; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nb {

// Predicted j-stream record of the FP64 path: 10 doubles = 80 bytes per body,
// {x, y, z, vx, vy, vz, ax, ay, az, m}, so that one tile of bodies is one
// contiguous block and a record is five 16-byte loads.
constexpr int kRecD = 10;
// Split-precision record: 16 floats = 64 bytes per body,
// {xh, yh, zh, m, xl, yl, zl, 0, vx, vy, vz, 0, ax, ay, az, 0}
// (x = xh + xl exactly to about 48 bits; v, a, m rounded to FP32).
constexpr int kRecF = 16;

// Device error words (one word per kind; kernels store 1, the host clears).
enum ErrWord : int { kErrIndex = 0, kErrNumeric = 1, kErrDtMin = 2, kErrLevel = 3, kErrWords = 4 };

// Small device block read back by the waiting calls.
struct Status {
    int64_t tick_next;
    int64_t n_act;
    double ekin;
    double epot;
    int32_t err[kErrWords];
    int64_t pad[2];
};

// Device arrays carved from the workspace.
struct Arrays {
    double *m, *x, *v, *a, *j, *s, *c, *a4n, *a5n, *phi;
    int64_t *tick;
    int32_t *level;
    double *jrec;      // [n][kRecD]
    float *jrec32;     // [n][kRecF] or nullptr
    double *evalbuf;   // [10][n]
    double *part;      // [10 * partial_slots]
    int32_t *act_idx;  // [n]
    int64_t *act_bmin; // [act_blocks]
    int32_t *act_bcnt; // [act_blocks]
    double *en_bsum;   // [2][en_blocks]
    Status *status;
    double *jrecj;     // [n][4] predicted jerks {jx, jy, jz, 0} (crackle evaluation)
    double *crk;       // [13][n] start-up crackle pass output, or nullptr
    unsigned *ectr;    // [kMaxGroups] group counters of the group kernel (zero between
                       // launches: each launch's last workgroup of a group resets its own)
};

// Launch shape of one evaluation.
struct EvalPlan {
    int ipl;     // active bodies per lane (1, 2); for the small-set and group kernels,
                 // minus the active bodies per wave (group kernel: per workgroup)
    int waves;   // waves per workgroup
    int tile;    // j-records per LDS tile (0: records read from memory directly)
    int jchunk;  // j-records per split (multiple of the tile, or of 64)
    int splits;  // number of j-splits S
    int iblocks; // workgroups along the active bodies (groups)
    int lw;      // small-set and group kernels: log2 of the lanes per active body; -1
                 // otherwise
    int fused;   // group kernel with S > 1: the last workgroup of a group adds the S
                 // partial slots (no separate reduction pass)
};

constexpr int kLaneTile = 64;     // records per LDS tile of the W-lanes-per-body sweeps
constexpr int kGroupTile = 256;   // records per LDS tile of the group kernel
constexpr int kMaxGroups = 1 << 16;  // group counters in a workspace
// The group kernel's in-launch reduction is used when the last workgroup of a group
// adds at most this many partial values per thread.
constexpr int kTailPerThread = 24;

constexpr int kActBS = 256;
constexpr int kActPerThread = 8;
constexpr int kActChunk = kActBS * kActPerThread;
constexpr int kEnBS = 256;

// ---- launchers (all asynchronous on `st`) ----
hipError_t launch_fill_f64(double *p, double v, size_t count, hipStream_t st);
hipError_t launch_fill_i64(int64_t *p, int64_t v, size_t count, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int32_t v, size_t count, hipStream_t st);
hipError_t launch_iota(int32_t *p, int64_t count, hipStream_t st);

hipError_t launch_predict(const Arrays &A, int64_t n, int64_t tick, int dt_min_log2,
                          bool split, hipStream_t st);
hipError_t launch_get_predicted(const Arrays &A, int64_t n, double *xp, double *vp, double *ap,
                                hipStream_t st);
hipError_t launch_copy_acc_to_jrec(const Arrays &A, int64_t n, bool split, hipStream_t st);
// j-records of n bodies from predicted [3][n] arrays and masses.
hipError_t launch_pack_records(const double *m, const double *xp, const double *vp,
                               const double *ap, int64_t n, double *jrec, hipStream_t st);
// out[0, count) = NaN if stt's index error word is set.
hipError_t launch_poison_on_index_error(const Status *stt, double *out, int64_t count,
                                        hipStream_t st);
hipError_t launch_start_store(const Arrays &A, int64_t n, hipStream_t st);

// One row of an evaluation launch table: the shape used for active sets of up to
// n_act_max bodies; target_waves sets the j-split count S ~ target / (waves along
// the active bodies).
struct EvalRow {
    int n_act_max, ipl, waves, tile, target_waves;
};
constexpr int kMaxEvalRows = 32;

// Shapes with a compiled kernel: ipl in {1, 2} with (waves, tile) in {(1, 64),
// (1, 128), (2, 128), (1, 256), (2, 256), (4, 256)} (a tile's 16-byte chunks split
// evenly); or, FP64 only, the small-set kernel: ipl = -Pmax (Pmax in {1, 2, 4, ..., 64}:
// at most Pmax active bodies per wave, each on 64 / P lanes with P = min(Pmax, the
// power of two >= n_act)), waves 1, tile 64 (LDS) or 0 (direct from memory).
// or, FP64 only, the group kernel (nbody_group.hip): ipl = -Pmax with Pmax in {1, 2,
// 4, ..., 64, 128} (the group's bodies; 128 = two per lane), waves 4 or 8, tile 256
// (LDS tiles; needs waves x 64 / Pmax <= 256) or 0 (direct reads).
bool eval_shape_supported(int ipl, int waves, int tile, bool split);
bool group_shape_ok(int pmax, int waves, int tile);
// Shape from a table (nrows == 0: the built-in table for the precision).
EvalPlan plan_eval(int64_t n, int64_t n_act, int64_t partial_slots, bool split,
                   const EvalRow *rows, int nrows);
// Shape with a fixed split count S (clamped to the number of tiles).
EvalPlan plan_eval_fixed(int64_t n, int64_t n_act, int ipl, int waves, int tile, int64_t S);
hipError_t launch_eval(const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                       int64_t n_act, double eps, bool split, double *out, hipStream_t st);
// The group kernel alone: with S > 1 it writes A.part and, when ctr is given (one
// zeroed counter per group), reduces them into dst (and dst2) itself.
hipError_t launch_eval_group(const Arrays &A, const EvalPlan &P, int64_t n, const int32_t *idx,
                             int64_t n_act, double eps, unsigned *ctr, double *dst, double *dst2,
                             hipStream_t st);

// Evaluation of every body against every body with each pair computed once
// (nbody_sym.hip): blocks of B bodies, a persistent grid of G workgroups claiming
// units (row block, part of a block) from a counter, partial sums in a row buffer and
// a column buffer (row_slots + col_slots doubles), then a fixed-order reduction into
// the index order. The geometry (and so the summation order) depends on n only.
constexpr int kSymWaves = 4;
constexpr int kSymGroups = 512;  // workgroups (fixed, so the summation order is too)
struct SymPlan {
    int B, nb, G, parts;  // block size, blocks, workgroups, parts per block
    int64_t units, row_slots, col_slots;
    // the last units are each cut into `fine` pieces: items (what workgroups claim)
    // 0 .. split0 - 1 are units 0 .. split0 - 1, then `fine` items per unit
    int fine;
    int64_t split0, items;
};
SymPlan plan_sym(int64_t n, int G);
hipError_t launch_eval_sym(const Arrays &A, const SymPlan &P, int64_t n, const int32_t *idx,
                           int64_t n_act, double eps, double *rowbuf, double *colbuf,
                           unsigned *claim, double *dst, double *dst2, hipStream_t st);

hipError_t launch_correct(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act,
                          int64_t tick, int dt_min_log2, hipStream_t st);
hipError_t launch_timesteps(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act,
                            int init, double eta, double eta_init, int dt_max_log2,
                            int dt_min_log2, hipStream_t st);
hipError_t launch_active(const Arrays &A, int64_t n, int L, int32_t *idx_out, hipStream_t st);
// Crackle evaluation (nbody_crackle.hip): predicts every body's jerk to `tick`,
// then a, j, s, crackle, phi of idx into out[13][n_act] (FP64).
hipError_t launch_eval_crackle(const Arrays &A, int64_t n, const int32_t *idx, int64_t n_act,
                               double eps, int64_t partial_slots, int64_t tick, int dt_min_log2,
                               double *out, hipStream_t st);
// c = rows 9..11 of the crackle output out[13][n] (every body; start-up).
hipError_t launch_store_crackle(const Arrays &A, int64_t n, const double *out, hipStream_t st);
hipError_t launch_energy(const Arrays &A, int64_t n, double eps, int64_t partial_slots,
                         hipStream_t st);

int act_blocks(int64_t n);
int en_blocks(int64_t n);

}  // namespace nb
