// kernels.hpp -- launchers of the GKR / sum-check kernels (kernels.hip).
//
// Every launcher enqueues on `st` and returns the launch status; none of
// them synchronises.  Device pointers only.  Reductions write one row of
// partial sums per workgroup into `partials`; a *_final kernel (one
// workgroup) folds the rows, writes the round message into the transcript,
// and only then draws the next challenge.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gkr {

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint8_t u8;

// Layer gate mix: the kernels drop the type array when a layer is uniform.
enum Kind { KIND_ADD = 0, KIND_MUL = 1, KIND_MIXED = 2 };

// Device state of an F2 sum-check.
struct ProofState {
    // SplitMix64 states of the challenge stream: the state before draw d
    // sits in rng[d & 1], so a launch reads one slot while its recorder
    // writes the other
    u64 rng[2];
    u64 pad[2];
};

// Workgroup size of every reduction kernel, and the cap on workgroups per
// launch (8 per CU on 256 CUs).
constexpr int BLOCK = 256;
constexpr int MAX_BLOCKS = 2048;

// Workgroups for n work items at `per` items per thread.
inline int blocks_for(u64 n, u64 per = 1) {
    u64 t = (n + per - 1) / per;
    u64 b = (t + BLOCK - 1) / BLOCK;
    if (b < 1) b = 1;
    if (b > (u64)MAX_BLOCKS) b = MAX_BLOCKS;
    return (int)b;
}

// ---- evaluation (a3) ------------------------------------------------------
hipError_t launch_load_inputs(hipStream_t st, const u64 *src, u32 S, u64 npad, u64 *V,
                              u32 *bad_flag);
// *bad_flag |= 1 if some src[g] >= p, g < n.
hipError_t launch_check_range(hipStream_t st, const u64 *src, u64 n, u32 *bad_flag);
// ---- proof bookkeeping ----------------------------------------------------
// eq half tables of a point pt[0..s): lo[x] = chi_x(pt[0..L)) for x < 2^L,
// hi[y] = chi_y(pt[L..s)) for y < 2^{s-L}; chi_x(pt) = lo[x & (2^L-1)] * hi[x >> L].
hipError_t launch_eq_halves(hipStream_t st, const u64 *pt, u32 s, u32 L, u64 *lo, u64 *hi);

// ---- verifier (a10) ---------------------------------------------------------
// Per workgroup (add~, mult~) partial sums at (a*, b*, c*) from half tables.
struct WiringArgs {
    int kind;
    u32 S;
    const u8 *type;
    const u32 *in1, *in2;
    const u64 *alo, *ahi;
    u32 La;
    const u64 *blo, *bhi;
    u32 Lb;
    const u64 *clo, *chi;
    u32 Lc;
    u64 *partials;
};
hipError_t launch_wiring(hipStream_t st, const WiringArgs &a, int *nblocks);
// Multilinear extension of T (n values, u64 or u32) at the point with half
// tables lo / hi (entry x weighs lo[x mod 2^L] hi[x >> L]): per-workgroup
// partial sums, stored, or added to the rows already there (accumulate), on
// nb_fixed workgroups (0: sized for n).  A chunk of a longer table starting
// at a multiple of 2^L passes hi advanced by its start >> L.
hipError_t launch_mle(hipStream_t st, u64 n, const u64 *T64, const u32 *T32, const u64 *lo,
                      const u64 *hi, u32 L, u64 *partials, int *nblocks, int accumulate = 0,
                      int nb_fixed = 0);
// Fold nparts rows of K partial sums into out[0..K).
hipError_t launch_reduce_rows(hipStream_t st, int nparts, int K, const u64 *partials, u64 *out);

// ---- F2 sum-check (a11) -------------------------------------------------------
// Round j over nm = n / 2^{j+1} pairs.  j = 0: pairs from the u32 vector.
// j = 1: fold the u32 vector by r_0 into Aout; j >= 2: fold Asrc (u64) by
// r_{j-1}, which every workgroup draws from the state round j-1 completed.
// Partials of round j: rows (sum A0^2, sum A1^2, sum (2 A1 - A0)^2) at
// part + 3 MAX_BLOCKS (j & 1).  For j >= 1 one more workgroup finishes round
// j-1: its message (G(0), G(1), G(2)) into prev_msg (and F2 = G(0) + G(1)
// into *f2 when not NULL), r_{j-1} into *prev_chal, and the state after it.
hipError_t launch_f2sc_round(hipStream_t st, int j, u64 nm, const u32 *a32, const u64 *Asrc,
                             u64 *Aout, ProofState *ps, u64 *part, int prev_parts, u64 *prev_msg,
                             u64 *prev_chal, u64 *f2, int *nblocks);
// The last rounds j0..l-1 in one workgroup, from level j0-1 of the table
// (u64, 2 F2SC_TAIL entries at most, stored by round j0-1's launch): it
// finishes round j0-1 (prev_parts rows), folds that level by r_{j0-1} into
// LDS, then per round sums the message, and only after a barrier that
// completes it draws the round's challenge and folds.  msgs and chals are
// the transcript's bases.  j0 >= 2.
constexpr int F2SC_TAIL = 4096;
hipError_t launch_f2sc_tail(hipStream_t st, int j0, int l, const u64 *Asrc, int prev_parts, const u64 *part,
                            ProofState *ps, u64 *msgs, u64 *chals);
// Finish of the last round j over its nparts partial rows, as above.
hipError_t launch_f2sc_final(hipStream_t st, int j, int nparts, const u64 *part, ProofState *ps,
                             u64 *msg, u64 *chal, u64 *f2);
hipError_t launch_f2sc_init(hipStream_t st, ProofState *ps, u64 seed);
// n == 1: the transcript is just F2 = a[0]^2.
hipError_t launch_f2sc_single(hipStream_t st, const u32 *a32, u64 *msg);

// ---- field check ----------------------------------------------------------
hipError_t launch_field_op(hipStream_t st, int op, const u64 *a, const u64 *b, u64 *out, u64 n);

}  // namespace gkr
