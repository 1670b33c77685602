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

// Device-resident protocol state of one proof.
struct ProofState {
    u64 rng;    // SplitMix64 state of the challenge stream
    u64 betaC;  // prod_{k<j} eq(z_k, r_k) while the a-variables are bound
    u64 v1;     // ~V_{i+1}(b*) once the b-variables are bound
    u64 pad;
};

// Workgroup size of every reduction kernel, and the cap on workgroups per
// launch (8 per CU on 256 CUs).
constexpr int BLOCK = 256;
constexpr int MAX_BLOCKS = 2048;
constexpr int MAX_LINE = 32;  // max number of line points t = 2..s' (s' <= 32)

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
hipError_t launch_eval(hipStream_t st, int kind, u32 S, u64 npad, const u8 *type, const u32 *in1,
                       const u32 *in2, const u64 *Vn, u64 *V);

// ---- proof bookkeeping ----------------------------------------------------
// rng = (seed << 8) | 2; draws z_0 (s0 values) into chals[0..s0) and zbuf;
// copies the S0 outputs into msgs[0..S0).
hipError_t launch_init_proof(hipStream_t st, ProofState *ps, u64 seed, u32 s0, const u64 *V0,
                             u32 S0, u64 *msgs, u64 *chals, u64 *zbuf);

// eq half tables of a point pt[0..s): lo[x] = chi_x(pt[0..L)) for x < 2^L,
// hi[y] = chi_y(pt[L..s)) for y < 2^{s-L}; chi_x(pt) = lo[x & (2^L-1)] * hi[x >> L].
hipError_t launch_eq_halves(hipStream_t st, const u64 *pt, u32 s, u32 L, u64 *lo, u64 *hi);

// ---- p-phase: the a-variables (a5) -----------------------------------------
// Round j over nm = 2^{s-j-1} pairs.  first: pairs from V (2^s values) and
// suffix weights B_0 from the z half tables, B_0 written to Bout.  Later
// rounds: fold Vsrc by r = *rptr into Vout (the round's pairs) and form
// B_j[m] = Bprev[2m] + Bprev[2m+1] into Bout (Bout may be NULL in the
// last round).  Partials: (sum B V[2m], sum B V[2m+1]).
hipError_t launch_pphase(hipStream_t st, bool first, u64 nm, const u64 *Vsrc, u64 *Vout,
                         const u64 *Bprev, u64 *Bout, const u64 *zlo, const u64 *zhi, u32 L,
                         const u64 *rptr, u64 *partials, int *nblocks);
// Message G(0) = C(1-z)S0, G(1) = C z S1, G(2) = C(3z-1)(2 S1 - S0) with
// C = ps->betaC, z = *zj; then r drawn into *chal; ps->betaC *= eq(z, r).
hipError_t launch_pfinal(hipStream_t st, int nparts, const u64 *partials, ProofState *ps,
                         const u64 *zj, u64 *msg, u64 *chal);

// ---- omega-phases: the b- and c-variables (a6, a8) -------------------------
// Round k of phase ph (1: bind in1 bits, 2: bind in2 bits) over S gates.
//   idx    wires bound in this phase (in1 for ph 1, in2 for ph 2)
//   oth    the other wires (in2 for ph 1, in1 for ph 2), read when init
//   F      V_{i+1} folded by the phase's earlier challenges (2^{s'-k} values)
//   Vn     V_{i+1} (ph 1 init reads the other operand from it)
//   a half tables of a*, b half tables of b* (ph 2 init)
//   rptr   challenge of round k-1 (unused when init)
//   w, off per-gate running weight and additive operand
// Partials: (E0, E1, O0, O1) = sums of w(F0+off), w(F1+off) over gates
// whose bit k is 0, resp. 1.
struct OmegaArgs {
    int kind, ph;
    bool init, write_w;
    u32 S, k;
    const u32 *idx, *oth;
    const u8 *type;
    const u64 *F, *Vn;
    const u64 *alo, *ahi;
    u32 La;
    const u64 *blo, *bhi;
    u32 Lb;
    const ProofState *ps;
    const u64 *rptr;
    u64 *w, *off;
    u64 *partials;
};
hipError_t launch_omega(hipStream_t st, const OmegaArgs &a, int *nblocks);
// Message G(0) = E0, G(1) = O1, G(2) = E0 - 2 E1 + 4 O1 - 2 O0; r drawn
// into *chal.  last = 1 / 2: this round ends phase 1 / 2, so the value
// Flast[0] + r (Flast[1] - Flast[0]) is v1 / v2: written to *vout (and
// ps->v1 for phase 1).
hipError_t launch_wfinal(hipStream_t st, int nparts, const u64 *partials, ProofState *ps, u64 *msg,
                         u64 *chal, int last, const u64 *Flast, u64 *vout);
// dst[m] = src[2m] + r (src[2m+1] - src[2m]) for m < nh, r = *rptr.
hipError_t launch_fold(hipStream_t st, u64 nh, const u64 *src, u64 *dst, const u64 *rptr);
// Layer i+1 has a single gate (s' = 0): v1 = v2 = Vn[0].
hipError_t launch_single_gate_end(hipStream_t st, const u64 *Vn, ProofState *ps, u64 *msg_v);

// ---- line step (a9) ---------------------------------------------------------
// T = s'-1 points l(t) = b* + t (c* - b*), t = 2..s'.  x = (hh 2^M + mid) 2^L
// + lane, chi_x(l(t)) = Hh_t[hh] Hl_t[mid] lo_t[lane]; L <= 6, 2^M waves.
// Tables: lo [T][2^L], hl [T][2^M], hh [2^{s'-L-M}][T].
hipError_t launch_line_tables(hipStream_t st, const u64 *bstar, const u64 *cstar, u32 sp, u32 L,
                              u32 M, u64 *lo, u64 *hl, u64 *hh);
// Partials per workgroup (rows of MAX_LINE): T sums of chi_x(l(t)) V[x].
hipError_t launch_line(hipStream_t st, u32 sp, u32 L, u32 M, const u64 *V, const u64 *lo,
                       const u64 *hl, const u64 *hh, u64 *partials, int *nblocks);
// h(t) for t = 2..s' into msg[0..T), tau drawn into *chal, z_{i+1} = l(tau)
// into zbuf; resets ps->betaC for the next layer.
hipError_t launch_line_final(hipStream_t st, int nparts, const u64 *partials, u32 sp,
                             ProofState *ps, const u64 *bstar, const u64 *cstar, u64 *msg,
                             u64 *chal, u64 *zbuf);

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
// Multilinear extension of T (n = 2^s values, u64 or u32) at the point with
// half tables lo / hi: per-workgroup partial sums.
hipError_t launch_mle(hipStream_t st, u64 n, const u64 *T64, const u32 *T32, const u64 *lo,
                      const u64 *hi, u32 L, u64 *partials, int *nblocks);
// Fold nparts rows of K partial sums into out[0..K).
hipError_t launch_reduce_rows(hipStream_t st, int nparts, int K, const u64 *partials, u64 *out);

// ---- F2 sum-check (a11) -------------------------------------------------------
// Round j over nm = n / 2^{j+1} pairs.  j = 0: pairs from the u32 vector.
// j = 1: fold the u32 vector by r into Aout; j >= 2: fold Asrc (u64).
// Partials: (sum A0^2, sum A1^2, sum (2 A1 - A0)^2).
hipError_t launch_f2sc_round(hipStream_t st, int j, u64 nm, const u32 *a32, const u64 *Asrc,
                             u64 *Aout, const u64 *rptr, u64 *partials, int *nblocks);
// Message (G(0), G(1), G(2)) into msg (and F2 = G(0) + G(1) into *f2 when
// not NULL), then r drawn into *chal.
hipError_t launch_f2sc_final(hipStream_t st, int nparts, const u64 *partials, ProofState *ps,
                             u64 *msg, u64 *chal, u64 *f2);
hipError_t launch_f2sc_init(hipStream_t st, ProofState *ps, u64 seed);
// n == 1: the transcript is just F2 = a[0]^2.
hipError_t launch_f2sc_single(hipStream_t st, const u32 *a32, u64 *msg);

// ---- field check ----------------------------------------------------------
hipError_t launch_field_op(hipStream_t st, int op, const u64 *a, const u64 *b, u64 *out, u64 n);

}  // namespace gkr
