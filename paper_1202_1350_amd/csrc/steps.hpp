// steps.hpp -- the prover as a program of steps, executed by one kernel.
//
// A proof is a fixed sequence of steps (evaluation of each layer, the
// circuit's first small layers whole in one step that also evaluates them,
// then per layer: the eq table of z, the p-phase rounds, the eq table of
// a*, the two omega-phases, the eq table of b*, and the line: V_{i+1}
// folded along it for layers of 2^11..2^22 entries, else the line points'
// eq tables and the line sums).  Most steps are one grid pass; a step that
// ends a sum-check round leaves one row of partial sums per workgroup.
//
// Every workgroup of the next step draws the round's challenge from the
// same SplitMix64 state (the verifier's coins do not depend on the
// messages), so no step ever synchronises workgroups inside a kernel; its
// workgroup 0 records the challenge and does the part of the round's finish
// that later rounds need (the beta prefix, v1 / v2, the next layer's z).
// Folding the rows into the message values is needed by nothing but the
// transcript, so every reducing step keeps rows of its own and one last
// step, ST_FINISH, folds all of them at once, one workgroup per message.
// The challenge of round j is drawn only in a launch that starts after the
// launch computing message j's sums has completed.
//
// One launch runs one step of each of several proofs (a job table maps
// workgroups to (proof, step)); a single proof is the one-job case.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gkr {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int32_t i32;
typedef uint8_t u8;

constexpr int SBLOCK = 512;      // threads per workgroup of the step kernel
constexpr int SMAX_BLOCKS = 512; // workgroups per step (2 per CU)
constexpr int LINE_CHUNK = 16;   // line points summed per workgroup
constexpr int ROW_STRIDE = 16;   // u64 per partial-sum row

enum StepKind : u32 {
    ST_EVAL = 0,   // V_i[g] = V_{i+1}[in1] op V_{i+1}[in2]
    ST_START,      // outputs into the transcript, z_0 drawn
    ST_EQ,         // eq half tables of a point (z_i suffix, a*, or b*)
    ST_P,          // one p-phase round (a-variables)
    ST_W,          // one omega round (b- or c-variables)
    ST_FOLD,       // fold of V_{i+1}'s table by the last challenge
    ST_LT,         // eq tables of the line points
    ST_LINE,       // line sums h(t), t = 2..s'
    ST_SGE,        // next layer has one gate: v1 = v2 = V_{i+1}[0]
    ST_END,        // nothing but the prologue
    ST_WAGG,       // omega phase, tables: per-gate weights summed by bound wire
    ST_WT0,        // omega phase, tables: level-0 tables and round 0
    ST_WT,         // omega phase, tables: round k >= 1 (fold, then sum)
    ST_WTAIL,      // omega phase, tables: remaining rounds in one workgroup
    ST_PTAIL,      // p-phase: remaining rounds in one workgroup
    ST_LOAD,       // inputs (pointer in state[3]) into V_d, range check
    ST_WA0,        // omega phase, tables: ST_WAGG and ST_WT0 in one pass, for
                   // layers whose wires each carry at most one chunk of gates
    ST_FINISH,     // every round's rows into its message values
    ST_WSMALL,     // omega phase of a small layer: eq table, level-0 tables, all rounds
    ST_TOP,        // the first layers whose tables all fit a tail, whole, in one workgroup
    ST_LFOLD,      // line of a wide layer: V_{i+1} folded along the line, 2^(tb+9) entries a workgroup
};

enum FinKind : u32 {
    FIN_NONE = 0,
    FIN_P,     // p-phase message from rows of (S0, S1)
    FIN_W,     // omega message from rows of (E0, E1, O0, O1)
    FIN_LINE,  // h(t) values from rows of line sums; then tau and z_{i+1}
    FIN_T,     // message (G(0), G(1), G(2)) from rows of three sums
    FIN_P2,    // two p-phase messages from rows of (S0, S1, U0, U1, W0, W1)
    FIN_T2,    // two table-round messages from rows of (G(0..2), Q0(0..2), Q1(0..2), Q2(0..2))
};

// Two rounds per launch.  The sums of round k+1 are, before r_k is known,
// polynomials in r_k with coefficients that are sums over the level-k
// tables: a step that reaches round k also sums those coefficients, and the
// finish of its rows writes message k, draws r_k, evaluates message k+1 at
// r_k, writes it and draws r_{k+1}.
//   p-phase: S0' = U0 + r_k U1, S1' = W0 + r_k W1.
//   table rounds: G'(t) = Q0(t) + r_k Q1(t) + r_k^2 Q2(t).

constexpr u32 KALL = 0xFFFF;  // kind resolved at run time (mixed batches)

// The finishes (bit f for FinKind f) a step of the given kind can carry;
// each kernel instantiation compiles only these.
__host__ __device__ constexpr u32 fin_mask(u32 kind) {
    return kind == KALL                              ? 0xFFu
           : kind == ST_P                            ? 1u << FIN_P2
           : kind == ST_PTAIL                        ? (1u << FIN_P) | (1u << FIN_P2) | (1u << FIN_LINE)
           : kind == ST_WT                           ? (1u << FIN_T) | (1u << FIN_T2)
           : kind == ST_WTAIL                        ? (1u << FIN_T) | (1u << FIN_T2)
           : kind == ST_EQ                           ? (1u << FIN_LINE) | (1u << FIN_W)
           : kind == ST_END                          ? 1u << FIN_LINE
           : (kind == ST_W || kind == ST_FOLD || kind == ST_LT || kind == ST_LFOLD) ? 1u << FIN_W
                                                     : 0u;
}

// Largest table (entries at the level a tail starts from, after its fold)
// that a one-workgroup tail keeps in LDS.
constexpr int TAIL_LIM = 1024;

// The point the ST_EQ step expands, assembled in LDS by each workgroup.
enum PointKind : u32 {
    PT_Z = 0,  // z_i[1..s): computed from the previous layer's line and tau
    PT_CHAL,   // challenges chals[base .. base+n) (the last may be drawn now)
};

// Per-proof device state shared by all steps of a proof.
struct ProofPtrs {
    u64 *msgs;   // transcript
    u64 *chals;  // challenges
    u64 *rngst;  // rngst[c] = SplitMix64 state before challenge c
    u64 *zbuf;   // z of the current layer
    u64 *state;  // [0] beta prefix C, [1] v1, [2] seed, [3] input pointer,
                 // [4] nonzero if an input is not below p
};

// Prologue: finish the previous round and/or draw challenge `draw`.  The
// message values themselves are written by ST_FINISH from `rows` (and, for
// p-phase rounds, the beta prefix and z values recorded in `rec`).
struct Fin {
    u32 kind;          // FinKind
    i32 draw;          // challenge index drawn here (-1: none)
    const u64 *rows;   // partial rows of the previous step
    u32 nrows;
    u64 *rec;          // FIN_P / FIN_P2: C, z_j (, z_{j+1}) at the time of the round
    u32 j;             // FIN_P: round index (z_j)
    u32 last;          // FIN_W: 1 / 2 = end of phase 1 / 2 (v1 / v2)
    u32 T;             // FIN_LINE: number of line values
    u32 sp;            // FIN_LINE: coordinates of z_{i+1}
    u32 chunk_blocks;  // FIN_LINE: workgroups per chunk of line points
    u32 ch;            // FIN_LINE: line points per chunk
    const u64 *F;      // FIN_W last: the 2-entry table
    u64 *msg;          // where the message goes
    u64 *vout;         // FIN_W last: transcript slot of v1 / v2
    const u64 *bstar, *cstar;  // FIN_LINE: line endpoints (chals)
};

// One message (or one chunk of line values) of ST_FINISH.
struct FinItem {
    u32 kind;          // FinKind
    u32 nrows;
    const u64 *rows;
    u64 *msg;
    const u64 *rec;    // FIN_P / FIN_P2
    i32 draw;          // FIN_P2 / FIN_T2: the challenge drawn after the first message
    u32 nvals;         // FIN_LINE: values of this chunk
};
struct FinishArgs {
    const FinItem *items;  // one per workgroup
    const u64 *chals;
};

struct EvalArgs {
    u32 kind, S;
    u64 npad;
    const u8 *type;
    const u32 *in1, *in2;
    const u64 *Vn;
    u64 *V;
};
struct LoadArgs {
    u32 S;
    u64 npad;
    u64 *V;
};
struct StartArgs {
    u32 s0, S0;
    const u64 *V0;
};
struct EqArgs {
    u32 point;  // PointKind
    u32 n;      // coordinates
    u32 L;      // lo table covers coordinates [0, L)
    u32 base;   // PT_CHAL: first challenge index; PT_Z: first coordinate of z
    u64 *lo, *hi;
    u32 beta_lo;  // a*: lo entries times beta(z, a*) (state[0]), so that a gate's
                  // weight beta chi_g(a*) is lo[g mod 2^L] hi[g >> L]
};
// p-phase grid step.  first: round 0 (and 1) on V_i and the eq tables of
// z_i[1..s); a unit is a quad of V_i (look) or a pair (s = 1); writes
// B_1 (look).  Otherwise: rounds j+2, j+3 from V^(j) and B_{j+1} folded by
// r_j, r_{j+1}; a unit is a quad of V^(j+2) (16 entries of V^(j), 4 of
// B_{j+1}); writes V^(j+2) and B_{j+3}.
struct PArgs {
    u32 first, look;
    u64 nu;        // units
    const u64 *Vsrc;
    u64 *Vout;
    const u64 *Bprev;
    u64 *Bout;
    const u64 *zlo, *zhi;
    u32 L;
};
struct WArgs {
    u32 kind, ph, init, write_w, inline_fold;
    u32 S, k;
    u64 nfold;
    const u32 *idx, *oth;
    const u8 *type;
    const u64 *F, *Vn;
    u64 *Fout;
    const u64 *alo, *ahi;
    u32 La;
    const u64 *blo, *bhi;
    u32 Lb;
    i32 rchal;  // non-inline rounds k > 0: index of r_{k-1} in chals
    u64 *w, *off;
};
struct FoldArgs {
    u64 nh;
    const u64 *src;
    u64 *dst;
};
struct LtArgs {
    u32 sp, L, M;
    u32 bbase, cbase;  // challenge indices of b* and c*
    u64 *lo, *hl, *hh;
};
// Line sums: chunk q of the workgroups takes points t' = q ch .. q ch + ch - 1
// (ch in {4, 8, 12, 16}, chunks of equal size); workgroups [q chunk_blocks,
// (q+1) chunk_blocks) make up a chunk.
struct LineArgs {
    u32 sp, L, M, T, chunk_blocks, ch;
    const u64 *V, *lo, *hl, *hh;
};
// Line of a layer with 2^11 <= 2^s' <= 2^32 by folding (ST_LFOLD):
// h(t) = ~V_{i+1}(b* + t (c* - b*)) is a polynomial of degree s' in t; V is
// folded coordinate by coordinate, each entry pair becoming a polynomial one
// degree higher.  With D = tb + 9, workgroup g (one per 2^D entries below
// S_{i+1}) folds entries [g 2^D, (g+1) 2^D) along coordinates 0..D-1 into
// a polynomial of degree D and writes its term of h(t), weighted along
// coordinates D..s'-1, for t = 2..s' as rows: value j in row
// (j / ROW_STRIDE) nwg + g, column j % ROW_STRIDE (nwg workgroups).
// ST_FINISH adds the rows up into h(2..s') as it does for the line sums'
// rows.
constexpr u32 LFOLD_MIN = 11, LFOLD_MAX = 32;
// Entries a thread folds, 2^tb: 128 to 256 workgroups from 2^17 to 2^22
// entries (a workgroup's time is set mostly by its LDS levels, not by tb), as
// many as there are below, and 2^(s' - 14) above (tb = 5 at most: more
// polynomials in registers would spill).
constexpr u32 lfold_tb(u32 sp) { return sp <= 17 ? 1 : sp == 18 ? 2 : sp <= 20 ? 3 : sp == 21 ? 4 : 5; }
static_assert(LFOLD_MIN >= 1 + 9, "a workgroup folds at least 2^(1 + 9) entries");
constexpr u32 lfold_wg(u32 sp) { return 1u << (sp - lfold_tb(sp) - 9); }
// Workgroups that cover the first n entries (V_{i+1} is zero from S_{i+1}
// on, so the blocks above hold zero polynomials and write no rows).
constexpr u32 lfold_wg_live(u32 sp, u64 n) {
    const u64 need = (n + (1ull << (lfold_tb(sp) + 9)) - 1) >> (lfold_tb(sp) + 9);
    return need < 1 ? 1u : need > lfold_wg(sp) ? lfold_wg(sp) : (u32)need;
}
constexpr u32 LFOLD_CHUNKS = 2;  // rows a workgroup: h(2..s'), s' - 1 <= 2 ROW_STRIDE values
static_assert(LFOLD_MAX - 1 <= LFOLD_CHUNKS * ROW_STRIDE, "h(2..s') fits a workgroup's rows");
static_assert(LFOLD_MAX <= 32, "b*_k and c*_k - b*_k of the line sit in 32 words of LDS each");
struct LfoldArgs {
    u32 sp, tb, bbase, cbase;  // coordinates; 2^tb entries a thread; challenge indices of b* and c*
    const u64 *V;              // V_{i+1}
    u64 *rows;                 // LFOLD_CHUNKS x nwg rows of ROW_STRIDE words
    const u64 *chals;
};
struct SgeArgs {
    const u64 *Vn;
    u64 *vslot;
};
// Tables of an omega phase: A[x] (weights) and C[x] (additive part) over
// the bound wire x, with F the fold of V_{i+1}:
//   G_k(t) = sum_m A_k(t, m) F_k(t, m) + C_k(t, m).
// Tiles of whole chunks spanning at most TILE_POS sorted positions (one
// wave each in the per-chunk sums), or a single big chunk of a heavy wire:
// tile t holds chunks [tch[t], tch[t+1]).
constexpr u32 TILE_POS = 64;
struct WaggArgs {
    u32 kind, ph;
    u32 nch;                 // chunks: sorted positions [cstart[ch], cstart[ch+1]) share one wire x
    const u32 *perm, *cstart;  // perm[p]: the gate at sorted position p
    const u32 *oths;         // other wire (ph 1: in2; ph 2: in1) by sorted position
    const u8 *types;         // gate type by sorted position (mixed layers)
    const u64 *Vn;
    const u64 *alo, *ahi;
    u32 La;
    const u64 *blo, *bhi;
    u32 Lb;
    u64 *partA, *partC;      // per chunk (ph 2: sums over ADD / MUL gates)
    u32 ntiles;              // tiles of whole chunks, at most 64 sorted positions each:
    const u32 *tch;          // tile t holds chunks [tch[t], tch[t+1])
};
struct Wt0Args {
    u32 ph, hasC;
    u64 npairs;
    const u32 *xch;          // chunks of wire x: [xch[x], xch[x+1])
    const u64 *partA, *partC;
    const u64 *F;            // V_{i+1}
    u64 *A, *C;              // level-0 tables
};
// ST_WA0: wire x's gates sit at sorted positions [rowptr[x], rowptr[x+1])
// (at most one chunk of gates per wire).
struct Wa0Args {
    u32 kind, ph, hasC;
    u64 npairs;
    const u32 *perm, *rowptr;
    const u32 *oths;
    const u8 *types;
    const u64 *Vn;           // V_{i+1}: gathered operands and the table F
    const u64 *alo, *ahi;
    u32 La;
    const u64 *blo, *bhi;
    u32 Lb;
    u64 *A, *C;              // level-0 tables
};
// Table step reading level k with pend (1 or 2) pending challenges: the
// tables folded to level k+pend, that round's sums and the next round's
// coefficients; a unit is a quad of level k+pend (4 << pend entries of
// level k).
struct WtArgs {
    u32 hasC, pend;
    u64 nu;
    const u64 *A, *C, *F;    // level k
    u64 *An, *Cn, *Fn;       // level k+pend
};
struct WtailArgs {
    u32 k0, sp, hasC, last;
    u32 pend;                // challenges the prologue drew (1 or 2): level k0 - pend is in memory
    u32 live;                // level-k0 entries [live, 2^{sp-k0}) are zero (not read)
    const u64 *A, *C, *F;    // level k0-pend, 2^{sp-k0+pend} entries
    u32 c0;                  // challenge index of round k0
    u64 *msg;                // message slot of round k0
    u64 *vout;
};
struct PtailArgs {
    u32 j0, s;
    u32 pend;                // challenges the prologue drew (1 or 2; 0 when j0 = 0)
    u32 live;                // entries [live, 2^{s-j0}) of V^(j0) are zero (not read)
    const u64 *V, *B;        // V^(j0-pend) (2^{s-j0+pend}) and B_{j0-1} (2^{s-j0});
                             // B NULL: B_{j0} is formed from z (j0 = 0, or the grid
                             // steps wrote B below the live entries only)
    u32 c0;                  // challenge index of round j0
    u64 *msg;                // message slot of round j0
};

// A small layer's whole omega phase in one workgroup: w as for ST_WA0
// (its eq table pointers are where this step writes the table of the
// phase's point), then rounds 0 .. sp-1 as a tail.
struct WsmallArgs {
    Wa0Args w;
    u32 eqn, eqL, eqbase;  // the point: coordinates, lo-table coordinates, challenge index
    u64 *eqlo, *eqhi;
    u32 sp, last, c0;       // last = phase (1: v1 into state[1]); c0: challenge index of round 0
    u64 *msg, *vout;
};

// ST_TOP: the sum-check of layers 0 .. nl-1 in one workgroup.  Every one of
// them has 2^s_i and 2^s_{i+1} (1 <= s_{i+1}) at most TAIL_LIM entries and
// one chunk of gates per wire in both omega phases.  Its p-phase, omega
// phases and line run as tails over tables kept in LDS from one layer to the
// next (V_{i+1}, read for the omega phases, is the next layer's V_i).
struct TopLayer {
    u32 s, sp, kind, co;       // s_i, s_{i+1}, gate mix, challenge index of round 0
    u64 *msg;                  // 3 n_i round values, v1, v2, h(2..s_{i+1})
    const u64 *Vn;             // V_{i+1}
    const u32 *rowptr[2], *perm[2], *oths[2];  // wire groups by in1 (phase 1) and in2 (phase 2)
    const u8 *types[2];        // gate types in sorted order (mixed layers)
    u32 S;                     // gates of layer i
    const u32 *in1, *in2;      // its wiring (evaluation)
    const u8 *type;            // its gate types (mixed layers)
    u64 *V;                    // V_i, written by the evaluation
};
// ST_TOP also evaluates its layers, nl - 1 down to 0, from V_nl (the layer
// below them, evaluated by ST_EVAL launches), and starts the proof as
// ST_START does (the randomness of z_0 and the outputs into the transcript).
struct TopArgs {
    u32 nl;
    const TopLayer *L;         // nl descriptors (device memory)
    const u64 *V0;             // V_0
};

struct StepDesc {
    u32 kind;
    u32 nblocks;
    u32 reduces;   // 1 if the step writes partial rows
    u32 K;         // values per row
    u64 *rows;     // this step's partial rows
    Fin fin;
    ProofPtrs pp;
    union {
        EvalArgs eval;
        StartArgs start;
        EqArgs eq;
        PArgs p;
        WArgs w;
        FoldArgs fold;
        LtArgs lt;
        LineArgs line;
        SgeArgs sge;
        WaggArgs wagg;
        Wt0Args wt0;
        WtArgs wt;
        WtailArgs wtail;
        PtailArgs ptail;
        LoadArgs load;
        Wa0Args wa0;
        FinishArgs finish;
        WsmallArgs wsmall;
        TopArgs top;
        LfoldArgs lfold;
    } u;
};

// One (proof, step) of a launch; workgroups [block0, next block0) run it.
struct JobEntry {
    const StepDesc *step;
    u32 block0;
    u32 pad;
};

// Workgroups a step needs.
u32 step_grid(const StepDesc &sd);
// One step of one proof (descriptor passed by value); ev0 / ev1 (or NULL)
// are recorded at the start and end of the dispatch.
hipError_t launch_step(hipStream_t st, const StepDesc &sd, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// One step of each of njobs proofs (entries in device memory, sorted by
// block0, followed by a sentinel whose block0 is the total; each job spans
// step_grid(*step) workgroups).
hipError_t launch_steps(hipStream_t st, const JobEntry *jobs, u32 njobs, u32 total_blocks,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// A launch's jobs passed by value (serving: the mix changes every launch).
constexpr int MAX_TABLE_JOBS = 128;
struct JobTable {
    u32 n, total;
    JobEntry e[MAX_TABLE_JOBS];
};
hipError_t launch_step_table(hipStream_t st, const JobTable &t);

// One proof of a batch: where its seed and input pointer go, and where its
// transcript is gathered.
struct BatchSlot {
    u64 *state;
    u64 seed, input;
    const u64 *msgs;
    u64 n_msgs, out_off, flag_off;
};
hipError_t launch_batch_setup(hipStream_t st, const BatchSlot *slots, u32 n);
hipError_t launch_batch_gather(hipStream_t st, const BatchSlot *slots, u32 n, u64 *out);

}  // namespace gkr
