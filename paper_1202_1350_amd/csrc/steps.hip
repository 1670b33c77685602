// steps.hip -- the step kernel: one launch runs one step of each job.
//
// Sec. 4.1.1 of the paper: every gate (or table entry) contributes
// independently to the prover's message, so a step is a grid-stride pass in
// which each workgroup sums its share (wave64 shuffles, then LDS) into one
// row of partial sums.  All arithmetic is exact in F_p (Sec. 6.1), so the
// result does not depend on the summation order.
#include <hip/hip_ext.h>

#include "fp61.hpp"
#include "steps.hpp"

namespace gkr {

using fp::add;
using fp::mul;
using fp::P;
using fp::sub;
using fp::u128;

struct alignas(16) u64x2 {
    u64 x, y;
};
__device__ __forceinline__ u64x2 ld2(const u64 *p, u64 i) { return *reinterpret_cast<const u64x2 *>(p + i); }
__device__ __forceinline__ void st2(u64 *p, u64 i, u64 a, u64 b) {
    u64x2 v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<u64x2 *>(p + i) = v;
}

constexpr int NWAVES = SBLOCK / 64;

// Data-parallel primitives moving one u64 as two 32-bit halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ u64 dpp64(u64 v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u32)v, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u32)(v >> 32), CTRL, ROWS, 0xf, true);
    return ((u64)(u32)hi << 32) | (u64)(u32)lo;
}
// Value of lane Q of this lane's quad (lanes 4m..4m+3).
template <int Q>
__device__ __forceinline__ u64 quad_get(u64 v) {
    return dpp64<Q | (Q << 2) | (Q << 4) | (Q << 6), 0xf>(v);
}

// Sum over the wave, left in lane 63: prefix sums within each row of 16
// lanes (shifts 1, 2, 4, 8), then row 0's total into row 1 and row 2's into
// row 3, then lane 31's into rows 2 and 3.  Lanes a shift leaves without a
// source read 0.
__device__ __forceinline__ u64 wave_sum63(u64 v) {
    v = add(v, dpp64<0x111, 0xf>(v));  // row_shr:1
    v = add(v, dpp64<0x112, 0xf>(v));  // row_shr:2
    v = add(v, dpp64<0x114, 0xf>(v));  // row_shr:4
    v = add(v, dpp64<0x118, 0xf>(v));  // row_shr:8
    v = add(v, dpp64<0x142, 0xa>(v));  // row_bcast:15 into rows 1, 3
    v = add(v, dpp64<0x143, 0xc>(v));  // row_bcast:31 into rows 2, 3
    return v;
}

// A value every lane holds the same copy of, moved to scalar registers.
__device__ __forceinline__ u64 uniform(u64 v) {
    const u32 lo = (u32)__builtin_amdgcn_readfirstlane((int)(u32)v);
    const u32 hi = (u32)__builtin_amdgcn_readfirstlane((int)(u32)(v >> 32));
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ u64 lane_value(u64 v, u32 l) {  // l uniform
    const u32 lo = (u32)__builtin_amdgcn_readlane((int)(u32)v, l);
    const u32 hi = (u32)__builtin_amdgcn_readlane((int)(u32)(v >> 32), l);
    return ((u64)hi << 32) | lo;
}

// Workgroup sum of v; thread k < K writes total k to out[k].
template <int K>
__device__ __forceinline__ void block_store(u64 (&v)[K], u64 *out) {
    __shared__ u64 sm[K][NWAVES];
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_sum63(v[k]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; k++) sm[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        u64 a = 0;
#pragma unroll
        for (int w = 0; w < NWAVES; w++) a = add(a, sm[threadIdx.x][w]);
        out[threadIdx.x] = a;
    }
    __syncthreads();
}

__device__ __forceinline__ u64 xor64(u64 v, int m) {
    const int lo = __shfl_xor((int)(u32)v, m), hi = __shfl_xor((int)(u32)(v >> 32), m);
    return ((u64)(u32)hi << 32) | (u64)(u32)lo;
}

// Sum rows [first, first + n) of K <= ROW_STRIDE values; every thread of the
// workgroup receives the totals.  Lane l of a wave reads column l % 16 of
// row l / 16, so one load brings four whole rows and the rows stream in as
// coalesced, independent loads (sixteen in flight per lane); the four
// lanes of a column are then summed across the wave and the waves in LDS.
template <int K>
__device__ __forceinline__ void rows_total(const u64 *rows, u32 first, u32 n, u64 (&tot)[K]) {
    static_assert(K <= ROW_STRIDE, "a row holds at most ROW_STRIDE values");
    constexpr u32 STEP = NWAVES * 4;  // rows per pass of the workgroup
    constexpr u32 U = 16;             // passes per batch of loads
    __shared__ u64 part[NWAVES][ROW_STRIDE];
    __shared__ u64 res[K];
    const u32 lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const u32 r0 = wid * 4 + (lane >> 4);
    const u64 *p = rows + ((u64)first + wid * 4) * ROW_STRIDE + lane;  // row first + r0, column lane % 16
    const u32 passes = r0 < n ? (n - r0 + STEP - 1) / STEP : 0;
    u64 acc[4] = {0, 0, 0, 0};
    for (u32 j = 0; j < passes; j += U) {  // a batch's loads are all issued before any add
        u64 x[U];
#pragma unroll
        for (int q = 0; q < (int)U; q++) x[q] = j + q < passes ? p[(u64)(j + q) * STEP * ROW_STRIDE] : 0;
#pragma unroll
        for (int q = 0; q < (int)U; q++) acc[q & 3] = add(acc[q & 3], x[q]);
    }
    u64 v = add(add(acc[0], acc[1]), add(acc[2], acc[3]));
    v = add(v, xor64(v, 16));
    v = add(v, xor64(v, 32));
    if (lane < (u32)K) part[wid][lane] = v;
    __syncthreads();
    if (threadIdx.x < (u32)K) {
        u64 t = part[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < NWAVES; w++) t = add(t, part[w][threadIdx.x]);
        res[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) tot[k] = res[k];
}

// chi of the bits of x over coordinates pt[0..n)
__device__ __forceinline__ u64 chi_bits(u64 x, const u64 *pt, u32 n) {
    u64 e = 1;
    for (u32 k = 0; k < n; k++) e = mul(e, fp::eqbit((u32)((x >> k) & 1), pt[k]));
    return e;
}

struct Ctx {
    u32 lb, nb;      // this workgroup within the step, workgroups of the step
    u64 gtid, gstride;
    u64 r;           // challenge drawn in the prologue
    u64 r2;          // the second one, after a two-round step
};

// What a tail takes over from its launch's prologue and finish: the RNG
// state after the drawn challenges (if the prologue drew any) and the beta
// prefix C (if the finish computed it, p-phase rounds).
struct TailIn {
    u64 st, C;
    u32 drew, have_c;
};

__device__ __forceinline__ u64 fold1(u64 x0, u64 x1, u64 r) {
    return fp::red128((u128)x0 + fp::wide(r, x1 + (fp::P - x0)));  // x1 - x0 + p < 2 p, unreduced
}

// fold1(fold1(x0, x1, r0), fold1(x2, x3, r0), r1) = x0 + r0 (x1 - x0) +
// r1 (x2 - x0) + r0 r1 ((x3 - x2) - (x1 - x0)), summed in 128 bits
// and reduced once; r01 = r0 r1.  Inputs canonical.
__device__ __forceinline__ u64 fold2(u64 x0, u64 x1, u64 x2, u64 x3, u64 r0, u64 r1, u64 r01) {
    // the differences unreduced: d1, d2 = x1 - x0 + p, x2 - x0 + p < 2 p and
    // d3 = x3 - x2 - x1 + x0 + 2 p < 4 p, so the sum stays below 8 p^2 + p < 2^125
    const u64 d1 = x1 + (fp::P - x0), d2 = x2 + (fp::P - x0), d3 = (x3 + x0) + (2 * fp::P - x1 - x2);
    return fp::red128((u128)x0 + fp::wide(r0, d1) + fp::wide(r1, d2) + fp::wide(r01, d3));
}

// Value t of a p-phase message from the two sums: G(0) = C (1-z) S0,
// G(1) = C z S1, G(2) = C (3z - 1)(2 S1 - S0); t is chosen per lane.
__device__ __forceinline__ u64 p_value(u32 t, u64 C, u64 z, u64 S0, u64 S1) {
    const u64 e = t == 0 ? sub(1, z) : (t == 1 ? z : sub(add(add(z, z), z), 1));
    const u64 S = t == 0 ? S0 : (t == 1 ? S1 : sub(add(S1, S1), S0));
    return mul(mul(C, e), S);
}

// Value k of tot, k chosen per lane.
template <int K>
__device__ __forceinline__ u64 pick(const u64 (&tot)[K], u32 k) {
    u64 v = 0;
#pragma unroll
    for (int q = 0; q < K; q++) v = k == (u32)q ? tot[q] : v;
    return v;
}

// The part of a round's finish that later rounds need; it reads no rows.
// Thread 0 records the beta prefix C and z of a p-phase round for its
// message, advances C by the drawn challenge(s) (left in *s_c as well), and
// at the end of an omega phase folds the last pair into v1 / v2; the line
// finish stores z_{i+1}.
template <u32 KIND>
__device__ __forceinline__ void fin_inline(const StepDesc &sd, const Ctx &c, const u64 *s_pt, u64 *s_c) {
    const Fin &f = sd.fin;
    const ProofPtrs &pp = sd.pp;
    constexpr u32 FM = fin_mask(KIND);
    const u32 tid = threadIdx.x;
    if ((FM & (1u << FIN_P)) && f.kind == FIN_P) {
        if (tid == 0) {
            const u64 z = pp.zbuf[f.j], C = pp.state[0];
            f.rec[0] = C;
            f.rec[1] = z;
            const u64 Cn = mul(C, fp::eq(z, c.r));  // beta prefix over r_0..r_j
            pp.state[0] = Cn;
            *s_c = Cn;
        }
    } else if ((FM & (1u << FIN_P2)) && f.kind == FIN_P2) {
        if (tid == 0) {
            const u64 z0 = pp.zbuf[f.j], z1 = pp.zbuf[f.j + 1], C = pp.state[0];
            f.rec[0] = C;
            f.rec[1] = z0;
            f.rec[2] = z1;
            const u64 Cn = mul(mul(C, fp::eq(z0, c.r)), fp::eq(z1, c.r2));
            pp.state[0] = Cn;
            *s_c = Cn;
        }
    } else if ((FM & (1u << FIN_W)) && f.kind == FIN_W) {
        if (f.last && tid == 0) {
            const u64 f0 = f.F[0], f1 = f.F[1];
            const u64 v = add(f0, mul(c.r, sub(f1, f0)));
            *f.vout = v;
            if (f.last == 1) pp.state[1] = v;
        }
    } else if ((FM & (1u << FIN_LINE)) && f.kind == FIN_LINE) {
        if (tid < f.sp) pp.zbuf[tid] = s_pt[tid];
        if (tid == 0) pp.state[0] = 1;  // the next layer's a-variables start unbound
    }
}

// One item of ST_FINISH: a round's rows into its message, lanes t < 3 (and
// 3..5 for a second message) writing one value each; operands that do not
// depend on the rows are loaded before the row sums.
__device__ __forceinline__ void step_finish(const FinishArgs &a, const Ctx &c) {
    const FinItem &it = a.items[c.lb];
    const u32 tid = threadIdx.x;
    switch (it.kind) {
        case FIN_P: {
            const u64 C = it.rec[0], z = it.rec[1];
            u64 t[2];
            rows_total<2>(it.rows, 0, it.nrows, t);
            if (tid < 3) it.msg[tid] = p_value(tid, C, z, t[0], t[1]);
            break;
        }
        case FIN_P2: {
            const u64 C = it.rec[0], z0 = it.rec[1], z1 = it.rec[2], r = a.chals[it.draw];
            u64 t[6];
            rows_total<6>(it.rows, 0, it.nrows, t);
            const u64 C1 = mul(C, fp::eq(z0, r));
            if (tid < 3) it.msg[tid] = p_value(tid, C, z0, t[0], t[1]);
            else if (tid < 6)
                it.msg[tid] = p_value(tid - 3, C1, z1, add(t[2], mul(r, t[3])), add(t[4], mul(r, t[5])));
            break;
        }
        case FIN_W: {
            u64 t[4];
            rows_total<4>(it.rows, 0, it.nrows, t);
            if (tid == 0) {
                const u64 E0 = t[0], E1 = t[1], O0 = t[2], O1 = t[3];
                it.msg[0] = E0;
                it.msg[1] = O1;
                u64 o4 = add(O1, O1);
                o4 = add(o4, o4);
                it.msg[2] = sub(add(sub(E0, add(E1, E1)), o4), add(O0, O0));
            }
            break;
        }
        case FIN_T: {
            u64 t[3];
            rows_total<3>(it.rows, 0, it.nrows, t);
            if (tid < 3) it.msg[tid] = pick(t, tid);
            break;
        }
        case FIN_T2: {
            const u64 r = a.chals[it.draw];
            u64 t[12];
            rows_total<12>(it.rows, 0, it.nrows, t);
            if (tid < 3) {
                it.msg[tid] = pick(t, tid);
            } else if (tid < 6) {  // round k+1 at t = tid - 3: Q0 + r (Q1 + r Q2)
                const u32 q = tid - 3;
                it.msg[tid] = add(pick(t, 3 + q), mul(r, add(pick(t, 6 + q), mul(r, pick(t, 9 + q)))));
            }
            break;
        }
        case FIN_LINE: {
            u64 t[LINE_CHUNK];
            rows_total<LINE_CHUNK>(it.rows, 0, it.nrows, t);
            if (tid < it.nvals) it.msg[tid] = pick(t, tid);
            break;
        }
        default: break;
    }
}

// ------------------------------------------------------------ step bodies

__device__ __forceinline__ void step_load(const LoadArgs &a, const ProofPtrs &pp, const Ctx &c) {
    const u64 *src = reinterpret_cast<const u64 *>(pp.state[3]);
    u64 bad = 0;
    for (u64 g = c.gtid; g < a.npad; g += c.gstride) {
        u64 v = 0;
        if (g < a.S) {
            v = src[g];
            bad |= v >= P;
        }
        a.V[g] = v;
    }
    if (bad) atomicOr(reinterpret_cast<unsigned long long *>(pp.state + 4), 1ull);
}

__device__ __forceinline__ void step_eval(const EvalArgs &a, const Ctx &c) {
    for (u64 g = c.gtid; g < a.npad; g += c.gstride) {
        u64 v = 0;
        if (g < a.S) {
            const u64 x = a.Vn[a.in1[g]], y = a.Vn[a.in2[g]];
            const bool ismul = a.kind == 1 || (a.kind == 2 && a.type[g]);
            v = ismul ? mul(x, y) : add(x, y);
        }
        a.V[g] = v;
    }
}

__device__ __forceinline__ void step_start(const StartArgs &a, const ProofPtrs &pp, const Ctx &c) {
    if (c.lb == 0 && threadIdx.x == 0) {
        u64 st = fp::sm_state(pp.state[2], fp::PURPOSE_GKR);  // state[2] = seed
        pp.rngst[0] = st;
        for (u32 k = 0; k < a.s0; k++) {
            const u64 z = fp::sm_field(st);
            pp.chals[k] = z;
            pp.zbuf[k] = z;
            pp.rngst[k + 1] = st;
        }
        pp.state[0] = 1;
        pp.state[1] = 0;
    }
    for (u64 g = c.gtid; g < a.S0; g += c.gstride) pp.msgs[g] = a.V0[g];
}

__device__ __forceinline__ void step_eq(const EqArgs &a, const Ctx &c, const u64 *pt, const ProofPtrs &pp) {
    const u64 nlo = 1ull << a.L, nhi = 1ull << (a.n - a.L);
    const u64 beta = a.beta_lo ? pp.state[0] : 1;
    for (u64 x = c.gtid; x < nlo + nhi; x += c.gstride) {
        if (x < nlo)
            a.lo[x] = a.beta_lo ? mul(beta, chi_bits(x, pt, a.L)) : chi_bits(x, pt, a.L);
        else
            a.hi[x - nlo] = chi_bits(x - nlo, pt + a.L, a.n - a.L);
    }
}

// x1 - x0 + p, not reduced (canonical x0, x1: below 2 p).
__device__ __forceinline__ u64 diff_lz(u64 x1, u64 x0) { return x1 + (fp::P - x0); }

// x mod p as red128 computes it, without the final subtraction: a value
// below p + 4 that is congruent to x.
__device__ __forceinline__ u64 red128_lz(u128 x) {
    const u64 lo = (u64)x, hi = (u64)(x >> 64);
    u64 s = (lo & fp::P) + (lo >> 61) + ((hi << 3) & fp::P) + (hi >> 58);  // < 2^63
    return (s & fp::P) + (s >> 61);
}

// Two-round steps give each quad (four consecutive entries of the level
// they sum over) to four adjacent lanes: lane j of the quad holds entry j,
// loads and stores stay coalesced, the quad's values are exchanged with DPP
// quad permutes and the quad's products are split over its lanes.

// p-phase quad v0..v3 of V^(j) with b0 = B_j[2u], b1 = B_j[2u+1]: round j's
// sums S0 = b0 v0 + b1 v2, S1 = b0 v1 + b1 v3 and the coefficients of round
// j+1's sums in r_j: U0 = bb v0, U1 = bb (v1 - v0), W0 = bb v2,
// W1 = bb (v3 - v2), bb = b0 + b1.  Lane j of the quad takes S0 (j = 0), S1
// (1), U0 and U1 (2), W0 and W1 (3): two products each, operands chosen by
// j so that all lanes run the same instructions.  x: its first (or only)
// sum, y: its second.
// bb and the differences stay unreduced (below 2 p), each product is
// reduced to below p + 4, and x, y are kept below p + 4 (canonical only
// when the step stores them).
__device__ __forceinline__ void p_quad(u32 j, u64 v0, u64 v1, u64 v2, u64 v3, u64 b0, u64 b1,
                                       u64 &x, u64 &y) {
    const u64 bb = b0 + b1;
    const bool s = j < 2;
    const u64 m1 = s ? b0 : bb, m2 = s ? b1 : bb;
    const u64 o1 = j == 0 ? v0 : (j == 1 ? v1 : (j == 2 ? v0 : v2));
    const u64 o2 = j == 0 ? v2 : (j == 1 ? v3 : (j == 2 ? diff_lz(v1, v0) : diff_lz(v3, v2)));
    const u64 p1 = red128_lz(fp::wide(m1, o1)), p2 = red128_lz(fp::wide(m2, o2));
    x = fp::fold64(x + (s ? p1 + p2 : p1));
    y = fp::fold64(y + (s ? 0 : p2));
}

// FIRST: whether this is the phase's first step, compile-time (1, 0; one
// kernel each) or -1 to take a.first.
template <int FIRST>
__device__ __forceinline__ void step_p(const PArgs &a, const Ctx &c, u64 *row) {
    const bool first = FIRST >= 0 ? FIRST != 0 : a.first != 0;
    const u64 mask = (1ull << a.L) - 1;
    auto beta0 = [&](u64 m) { return mul(a.zlo[m & mask], a.zhi[m >> a.L]); };  // B_0[m]
    if (first && !a.look) {
        // one round (s = 1)
        u64 acc[2] = {0, 0};
        for (u64 m = c.gtid; m < a.nu; m += c.gstride) {
            const u64x2 p = ld2(a.Vsrc, 2 * m);
            const u64 b = beta0(m);
            acc[0] = add(acc[0], mul(b, p.x));
            acc[1] = add(acc[1], mul(b, p.y));
        }
        block_store<2>(acc, row);
        return;
    }
    u64 x = 0, y = 0;  // this lane's sums (see p_quad)
    const u64 r0 = c.r, r1 = c.r2, r01 = mul(r0, r1);
    // lanes g = 4u + j; the stride is a multiple of 4, so a quad's lanes
    // leave the loop together
    for (u64 g = c.gtid; (g >> 2) < a.nu; g += c.gstride) {
        const u64 u = g >> 2;
        const u32 j = (u32)(g & 3);
        u64 v, bq;  // entry 4u + j of this step's level; B of that level at pair 2u + j/2
        if (first) {
            v = a.Vsrc[g];
            bq = beta0(2 * u + (j >> 1));  // lanes 0, 1: B_0[2u]; lanes 2, 3: B_0[2u+1]
        } else {
            const u64x2 p = ld2(a.Vsrc, 4 * g), q = ld2(a.Vsrc, 4 * g + 2);
            v = fold2(p.x, p.y, q.x, q.y, r0, r1, r01);
            if (a.Vout) a.Vout[g] = v;
            bq = a.Bprev[g];  // B_{j+1}[4u + j]
        }
        const u64 v0 = quad_get<0>(v), v1 = quad_get<1>(v), v2 = quad_get<2>(v), v3 = quad_get<3>(v);
        u64 b0, b1;
        if (first) {
            b0 = quad_get<0>(bq);
            b1 = quad_get<2>(bq);
        } else {
            b0 = add(quad_get<0>(bq), quad_get<1>(bq));  // B_{j+2}[2u]
            b1 = add(quad_get<2>(bq), quad_get<3>(bq));  // B_{j+2}[2u+1]
        }
        if (j == 0 && a.Bout) a.Bout[u] = add(b0, b1);
        p_quad(j, v0, v1, v2, v3, b0, b1, x, y);
    }
    // rows: S0, S1, U0, U1, W0, W1
    x = fp::canon(x);
    y = fp::canon(y);
    const u32 j = (u32)(c.gtid & 3);
    u64 acc[6] = {j == 0 ? x : 0, j == 1 ? x : 0, j == 2 ? x : 0, j == 2 ? y : 0, j == 3 ? x : 0,
                  j == 3 ? y : 0};
    block_store<6>(acc, row);
}

// Gate g with bound-wire index idx, at round k of its phase:
//   term_g(t) = w_g eq(bit_k(idx), t) (F(t) + off_g)
// with F(t) = (1-t) F[2m] + t F[2m+1], m = idx >> (k+1), the extension of
// V_{i+1} at the partially bound point.  MUL gates carry their fixed
// operand inside w (off = 0), ADD gates in off.  With P0 = w (F[2m] + off),
// P1 = w (F[2m+1] + off):  bit 0 adds P0 at t=0 and P0 - 2 P1 at t=2;
// bit 1 adds P1 at t=1 and 4 P1 - 2 P0 at t=2.  The row holds (E0, E1)
// = sums of (P0, P1) over bit-0 gates and (O0, O1) over bit-1 gates.
template <int KIND, int PH>
__device__ __forceinline__ void step_w(const WArgs &a, const Ctx &c, const ProofPtrs &pp, u64 *row) {
    const bool init = a.init, inl = a.inline_fold, wr = a.write_w;
    u64 r = 0, omr = 0;
    if (!init) {
        r = inl ? c.r : pp.chals[a.rchal];
        omr = sub(1, r);
    }
    const u64 v1 = PH == 2 ? pp.state[1] : 0;
    const u64 amask = (1ull << a.La) - 1, bmask = (1ull << a.Lb) - 1;
    const u32 k = a.k;
    if (inl) {
        // this round's table F^(k) = F^(k-1) folded by r, for the next round
        for (u64 m = c.gtid; m < a.nfold; m += c.gstride) {
            const u64x2 p = ld2(a.F, 2 * m);
            a.Fout[m] = add(p.x, mul(r, sub(p.y, p.x)));
        }
    }
    u64 acc[4] = {0, 0, 0, 0};
    for (u64 g = c.gtid; g < a.S; g += c.gstride) {
        const u32 idx = a.idx[g];
        const bool ismul = KIND == 1 || (KIND == 2 && a.type[g]);
        u64 wt, of;
        if (init) {
            u64 wg = mul(a.alo[g & amask], a.ahi[g >> a.La]);  // beta chi_g(a*): lo carries beta
            if (PH == 1) {
                const u64 y = a.Vn[a.oth[g]];
                wt = ismul ? mul(wg, y) : wg;
                of = ismul ? 0 : y;
                if (KIND != 1) a.off[g] = of;
            } else {
                const u32 i1 = a.oth[g];
                wg = mul(wg, mul(a.blo[i1 & bmask], a.bhi[i1 >> a.Lb]));
                wt = ismul ? mul(wg, v1) : wg;
                of = ismul ? 0 : v1;
            }
        } else {
            wt = mul(a.w[g], ((idx >> (k - 1)) & 1) ? r : omr);
            if (PH == 1)
                of = KIND == 1 ? 0 : a.off[g];
            else
                of = ismul ? 0 : v1;
        }
        u64 f0, f1;
        if (inl) {
            const u64 q = ((u64)idx >> (k + 1)) << 2;
            const u64x2 p0 = ld2(a.F, q), p1 = ld2(a.F, q + 2);
            f0 = add(p0.x, mul(r, sub(p0.y, p0.x)));
            f1 = add(p1.x, mul(r, sub(p1.y, p1.x)));
        } else {
            const u64x2 f = ld2(a.F, ((u64)idx >> (k + 1)) << 1);
            f0 = f.x;
            f1 = f.y;
        }
        const u64 P0 = mul(wt, add(f0, of)), P1 = mul(wt, add(f1, of));
        if ((idx >> k) & 1) {
            acc[2] = add(acc[2], P0);
            acc[3] = add(acc[3], P1);
        } else {
            acc[0] = add(acc[0], P0);
            acc[1] = add(acc[1], P1);
        }
        if (wr) a.w[g] = wt;
    }
    block_store<4>(acc, row);
}

__device__ __forceinline__ void step_fold(const FoldArgs &a, const Ctx &c) {
    const u64 r = c.r;
    for (u64 m = c.gtid; m < a.nh; m += c.gstride) {
        const u64x2 p = ld2(a.src, 2 * m);
        a.dst[m] = add(p.x, mul(r, sub(p.y, p.x)));
    }
}

// Line step (a9).  h(t) = ~V_{i+1}(l(t)) for t = 2..s', l(t) = b* + t (c* - b*).
// x = (hh 2^M + mid) 2^L + lane: chi_x(l(t)) = Hh_t[hh] Hl_t[mid] lo_t[lane].
// Tables: lo [T][2^L], hl [T][2^M], hh [2^H][T].
__device__ __forceinline__ void step_lt(const LtArgs &a, const Ctx &c, const u64 *bstar, const u64 *cstar) {
    if (a.sp < 2) return;  // no line points
    const u32 T = a.sp - 1, H = a.sp - a.L - a.M;
    const u64 nlo = 1ull << a.L, nhl = 1ull << a.M, nhh = 1ull << H;
    const u64 per = nlo + nhl + nhh;
    for (u64 e = c.gtid; e < (u64)T * per; e += c.gstride) {
        const u32 tp = (u32)(e / per);
        const u64 x = e % per;
        const u64 t = tp + 2;
        u32 base, n;
        u64 bits;
        if (x < nlo) {
            base = 0; n = a.L; bits = x;
        } else if (x < nlo + nhl) {
            base = a.L; n = a.M; bits = x - nlo;
        } else {
            base = a.L + a.M; n = H; bits = x - nlo - nhl;
        }
        u64 v = 1;
        for (u32 k = 0; k < n; k++) {
            const u64 b = bstar[base + k], cc = cstar[base + k];
            const u64 l = add(b, mul(t, sub(cc, b)));
            v = mul(v, fp::eqbit((u32)((bits >> k) & 1), l));
        }
        if (x < nlo)
            a.lo[(u64)tp * nlo + bits] = v;
        else if (x < nlo + nhl)
            a.hl[(u64)tp * nhl + bits] = v;
        else
            a.hh[bits * T + tp] = v;
    }
}

// Workgroups [q * chunk_blocks, (q+1) * chunk_blocks) sum line points
// t' = 16 q .. 16 q + 15; within a chunk, wave `mid` walks hh.
// The weights hh[h][t] of 64 consecutive h pass through LDS (one read per
// tile, broadcast reads in the loop); every lane runs the loop, lanes past
// the table adding zeros.  Products are summed exactly in 128 bits and
// reduced once per tile (<= 64 terms).
template <int CH>
__device__ void line_sums(const LineArgs &a, const Ctx &c, u64 *row) {
    __shared__ u64 s_w[64][CH];
    const u32 T = a.T, H = a.sp - a.L - a.M;
    const u64 nlo = 1ull << a.L, nhl = 1ull << a.M, nhh = 1ull << H;
    const u32 chunk = c.lb / a.chunk_blocks;
    const u32 t0 = chunk * CH;
    const u32 lane = threadIdx.x & 63;
    const u64 mid = (u64)(c.lb - chunk * a.chunk_blocks) * NWAVES + (threadIdx.x >> 6);
    const bool ok = lane < nlo && mid < nhl;
    const u64 x0 = ok ? (mid << a.L) + lane : 0;
    u64 s[CH];
#pragma unroll
    for (int t = 0; t < CH; t++) s[t] = 0;
    for (u64 h0 = 0; h0 < nhh; h0 += 64) {
        const u32 nh = nhh - h0 < 64 ? (u32)(nhh - h0) : 64u;
        __syncthreads();  // the previous tile's weights are read
        for (u32 i = threadIdx.x; i < 64u * CH; i += SBLOCK) {
            const u32 hl = i / CH, t = i % CH;
            s_w[hl][t] = hl < nh && t0 + t < T ? a.hh[(h0 + hl) * T + t0 + t] : 0;
        }
        __syncthreads();
        u128 w128[CH];
#pragma unroll
        for (int t = 0; t < CH; t++) w128[t] = s[t];
        for (u32 hl = 0; hl < nh; hl++) {
            const u64 v = ok ? a.V[((h0 + hl) << (a.M + a.L)) + x0] : 0;
#pragma unroll
            for (int t = 0; t < CH; t++) w128[t] += fp::wide(s_w[hl][t], v);
        }
#pragma unroll
        for (int t = 0; t < CH; t++) s[t] = fp::red128(w128[t]);
    }
    u64 acc[LINE_CHUNK];
#pragma unroll
    for (int t = 0; t < LINE_CHUNK; t++) {
        acc[t] = 0;
        if (t < CH && t0 + t < T && ok)
            acc[t] = mul(s[t < CH ? t : 0], mul(a.hl[(u64)(t0 + t) * nhl + mid], a.lo[(u64)(t0 + t) * nlo + lane]));
    }
    block_store<LINE_CHUNK>(acc, row);
}

__device__ __forceinline__ void step_line(const LineArgs &a, const Ctx &c, u64 *row) {
    switch (a.ch) {
        case 4: line_sums<4>(a, c, row); break;
        case 8: line_sums<8>(a, c, row); break;
        case 12: line_sums<12>(a, c, row); break;
        default: line_sums<16>(a, c, row); break;
    }
}

// ------------------------------------------- omega phases over tables
//
// Grouping the gates of an omega phase by the wire x they bind, the
// per-gate terms w_g eq(bit_k(x), t) (F(t) + off_g) of round k sum to
//   G_k(t) = sum_m A_k(t, m) F_k(t, m) + C_k(t, m),
// with A_0[x] = sum of w_g over the gates on x, C_0[x] = sum of w_g off_g,
// and A_k, C_k, F_k the folds of A_0, C_0 and V_{i+1} by the phase's first
// k challenges (all three are multilinear in the bound bits).  The gates are
// read once per phase instead of once per round.

// Sums over the gates perm[p0 .. p1) of one wire x.  Phase 1: MUL gates
// put w V[in2] on x's value (sA), ADD gates put w on it (sA) and add
// w V[in2] (sC).  Phase 2: sums of the weights over ADD gates (sA) and MUL
// gates (sC); v1 enters when the level-0 tables are formed.
// GK, PH: the layer's gate mix (0 ADD, 1 MUL, 2 mixed) and the phase when
// known at compile time, -1 and 0 to read them from a.
template <int GK = -1, int PH = 0, typename Args>
__device__ __forceinline__ void wire_sums(const Args &a, u32 p0, u32 p1, u64 &sA_out, u64 &sC_out) {
    const u32 kind = GK >= 0 ? (u32)GK : a.kind, ph = PH > 0 ? (u32)PH : a.ph;
    const u64 amask = (1ull << a.La) - 1, bmask = (1ull << a.Lb) - 1;
    // branch-free updates keep both sums in registers; a sum that a gate
    // mix leaves at zero is not updated
    u64 sA = 0, sC = 0;
    for (u32 p = p0; p < p1; p++) {
        const u32 g = a.perm[p], o = a.oths[p];
        const bool ismul = kind == 1 || (kind == 2 && a.types[p]);
        u64 w = mul(a.alo[g & amask], a.ahi[g >> a.La]);  // beta chi_g(a*): lo carries beta
        if (ph == 1) {
            const u64 wy = mul(w, a.Vn[o]);
            if (kind == 1) {
                sA = add(sA, wy);
            } else {
                sA = add(sA, ismul ? wy : w);
                sC = add(sC, ismul ? 0 : wy);
            }
        } else {
            const u32 i1 = o;
            w = mul(w, mul(a.blo[i1 & bmask], a.bhi[i1 >> a.Lb]));
            if (kind == 1) {
                sC = add(sC, w);
            } else if (kind == 0) {
                sA = add(sA, w);
            } else {
                sA = add(sA, ismul ? 0 : w);
                sC = add(sC, ismul ? w : 0);
            }
        }
    }
    sA_out = sA;
    sC_out = sC;
}

// Value v of lane l (l uniform or not; every lane of the wave takes part).
__device__ __forceinline__ u64 bperm64(u64 v, u32 l) {
    const int lo = __builtin_amdgcn_ds_bpermute((int)(l << 2), (int)(u32)v);
    const int hi = __builtin_amdgcn_ds_bpermute((int)(l << 2), (int)(u32)(v >> 32));
    return ((u64)(u32)hi << 32) | (u64)(u32)lo;
}

// Per-chunk sums of the gates' terms (wires with more than one chunk).  A
// wave takes a tile of whole chunks (at most 64 sorted positions) and lane
// l the gate at the tile's position l, so the gate arrays are read in
// coalesced runs; the inclusive scan of the terms over the wave gives each
// chunk's sum as the scan at its last position minus the scan just before
// its first.  Terms as in wire_sums (beta(z, a*), which multiplies every
// term, comes with the lo half of a*'s eq table).
// GK, PH: the gate mix and phase, compile-time (one kernel each) or -1, 0.
template <int GK, int PH>
__device__ __forceinline__ void step_wagg(const WaggArgs &a, const ProofPtrs &pp, const Ctx &c) {
    (void)pp;  // beta(z, a*) is in the lo half of a*'s eq table
    const u32 kind = GK >= 0 ? (u32)GK : a.kind, ph = PH > 0 ? (u32)PH : a.ph;
    const u32 lane = threadIdx.x & 63;
    const u64 amask = (1ull << a.La) - 1, bmask = (1ull << a.Lb) - 1;
    const u64 nwaves = c.gstride >> 6;
    for (u64 t = c.gtid >> 6; t < a.ntiles; t += nwaves) {  // wave-uniform
        const u32 c0 = a.tch[t], nc = a.tch[t + 1] - c0;
        if (nc == 0) continue;  // (a group without gates has one empty tile)
        const u32 base = a.cstart[c0], end = a.cstart[c0 + nc];
        if (end - base > TILE_POS) {  // one big chunk of a heavy wire: lanes stride over it
            u64 sA = 0, sC = 0;
#pragma unroll 4
            for (u32 q = base + lane; q < end; q += 64) {
                const u32 g = a.perm[q], o = a.oths[q];
                const bool ismul = kind == 1 || (kind == 2 && a.types[q]);
                u64 w = mul(a.alo[g & amask], a.ahi[g >> a.La]);
                if (ph == 1) {
                    const u64 wy = mul(w, a.Vn[o]);
                    sA = add(sA, ismul ? wy : w);
                    sC = add(sC, ismul ? 0 : wy);
                } else {
                    w = mul(w, mul(a.blo[o & bmask], a.bhi[o >> a.Lb]));
                    sA = add(sA, ismul ? 0 : w);
                    sC = add(sC, ismul ? w : 0);
                }
            }
            sA = wave_sum63(sA);
            sC = wave_sum63(sC);
            if (lane == 63) {
                a.partA[c0] = sA;
                a.partC[c0] = sC;
            }
            continue;
        }
        const u32 p = base + lane;
        u64 vA = 0, vC = 0;
        if (p < end) {
            const u32 g = a.perm[p], o = a.oths[p];
            const bool ismul = kind == 1 || (kind == 2 && a.types[p]);
            u64 w = mul(a.alo[g & amask], a.ahi[g >> a.La]);
            if (ph == 1) {
                const u64 wy = mul(w, a.Vn[o]);
                vA = ismul ? wy : w;
                vC = ismul ? 0 : wy;
            } else {
                w = mul(w, mul(a.blo[o & bmask], a.bhi[o >> a.Lb]));
                vA = ismul ? 0 : w;
                vC = ismul ? w : 0;
            }
        }
        const u64 sA = wave_sum63(vA), sC = wave_sum63(vC);  // inclusive scans
        const bool mine = lane < nc;  // lane k writes chunk c0 + k
        const u32 k = mine ? lane : 0;
        const u32 first = a.cstart[c0 + k] - base, last = a.cstart[c0 + k + 1] - base - 1;
        const u32 before = first ? first - 1 : 0;
        const u64 A1 = bperm64(sA, last), C1 = bperm64(sC, last);
        const u64 A0 = bperm64(sA, before), C0 = bperm64(sC, before);
        if (mine) {
            a.partA[c0 + k] = first ? sub(A1, A0) : A1;
            a.partC[c0 + k] = first ? sub(C1, C0) : C1;
        }
    }
}

// Message sums of one pair of a table round.  HC: whether the layer has a
// C table, when known at compile time (without one C is zero and skipped).
template <int HC = 1>
__device__ __forceinline__ void table_terms(u64 A0, u64 A1, u64 C0, u64 C1, u64 F0, u64 F1,
                                            u64 (&acc)[3]) {
    const u64 A2 = sub(add(A1, A1), A0), F2 = sub(add(F1, F1), F0);
    if (HC) {
        const u64 C2 = sub(add(C1, C1), C0);
        acc[0] = add(acc[0], add(mul(A0, F0), C0));
        acc[1] = add(acc[1], add(mul(A1, F1), C1));
        acc[2] = add(acc[2], add(mul(A2, F2), C2));
    } else {
        acc[0] = add(acc[0], mul(A0, F0));
        acc[1] = add(acc[1], mul(A1, F1));
        acc[2] = add(acc[2], mul(A2, F2));
    }
}

// One quad of level-k tables, held one entry per lane by four adjacent
// lanes.  Lane t < 3 adds, for its t, round k's value over the quad's two
// pairs and round k+1's three coefficients (lane 3's sums are dropped): the quad
// folds to the pair (X0 + r dX0, X2 + r dX2), dX0 = X1 - X0, dX2 = X3 - X2,
// whose value at t is a_t + r b_t with a = (X0, X2, 2 X2 - X0),
// b = (dX0, dX2, 2 dX2 - dX0):
//   Q0(t) += aA aF + aC, Q1(t) += aA bF + bA aF + bC, Q2(t) += bA bF.
// Every lane runs the same instructions (operands chosen by t), so a wave
// does six products per quad.  acc: G(t), Q0(t), Q1(t), Q2(t) of this lane.
struct QuadAcc {
    u64 g = 0, q0 = 0, q1 = 0, q2 = 0;
};


// x at t in {0, 1, 2} on the line through (0, x0), (1, x1), not reduced:
// with x0, x1 < K p the value is below 3 K p (K <= 2: below 2^64).  It only
// feeds 128-bit product sums, which red128 reduces whatever their size.
template <int K>
__device__ __forceinline__ u64 at_t_lz(u64 x0, u64 x1, u32 t) {
    static_assert(K == 1 || K == 2, "3 K p < 2^64");
    const u64 x2 = 2 * x1 + ((u64)K * fp::P - x0);
    return t == 0 ? x0 : (t == 1 ? x1 : x2);
}

// HC: whether the layer has a C table (1, 0), or -1 to take hasC.  The line
// values and differences stay unreduced (below 6 p); each of g, q0, q1, q2
// is one 128-bit sum of at most two products and two such values, reduced
// once (below 2^128: 2 (3p)(6p) + 9p < 2^127.3).
template <int HC>
__device__ __forceinline__ void table_quad(u32 j, u64 A, u64 C, u64 F, bool hasC, QuadAcc &acc) {
    const bool hc = HC >= 0 ? HC != 0 : hasC;
    const u64 A0 = quad_get<0>(A), A1 = quad_get<1>(A), A2 = quad_get<2>(A), A3 = quad_get<3>(A);
    const u64 F0 = quad_get<0>(F), F1 = quad_get<1>(F), F2 = quad_get<2>(F), F3 = quad_get<3>(F);
    u64 C0 = 0, C1 = 0, C2 = 0, C3 = 0;
    if (hc) {
        C0 = quad_get<0>(C);
        C1 = quad_get<1>(C);
        C2 = quad_get<2>(C);
        C3 = quad_get<3>(C);
    }
    const u32 t = j < 3 ? j : 2;
    // round k at t: pairs (X0, X1) and (X2, X3)
    u128 gs = fp::wide(at_t_lz<1>(A0, A1, t), at_t_lz<1>(F0, F1, t)) +
              fp::wide(at_t_lz<1>(A2, A3, t), at_t_lz<1>(F2, F3, t));
    if (HC != 0) gs += (u128)at_t_lz<1>(C0, C1, t) + at_t_lz<1>(C2, C3, t);  // (zero without a C table)
    // round k+1's coefficients at t
    const u64 aA = at_t_lz<1>(A0, A2, t), bA = at_t_lz<2>(diff_lz(A1, A0), diff_lz(A3, A2), t);
    const u64 aF = at_t_lz<1>(F0, F2, t), bF = at_t_lz<2>(diff_lz(F1, F0), diff_lz(F3, F2), t);
    u128 s0 = fp::wide(aA, aF), s1 = fp::wide(aA, bF) + fp::wide(bA, aF);
    if (HC != 0) {
        s0 += at_t_lz<1>(C0, C2, t);
        s1 += at_t_lz<2>(diff_lz(C1, C0), diff_lz(C3, C2), t);
    }
    const u64 g = red128_lz(gs), q0 = red128_lz(s0), q1 = red128_lz(s1), q2 = red128_lz(fp::wide(bA, bF));
    // sums kept below p + 4 (lane 3's are never stored, see table_quad_store)
    acc.g = fp::fold64(acc.g + g);
    acc.q0 = fp::fold64(acc.q0 + q0);
    acc.q1 = fp::fold64(acc.q1 + q1);
    acc.q2 = fp::fold64(acc.q2 + q2);
}

// Rows of a two-round table step: G(0..2), Q0(0..2), Q1(0..2), Q2(0..2);
// lane t contributes slot t of each.
// The workgroup's row: G(t), Q0(t), Q1(t), Q2(t) at t, 3 + t, 6 + t, 9 + t.
// Lane j of every quad holds t = j, so lanes of equal j are summed: row
// shifts by 4 and 8 leave a row's sums in its lanes 12 + j, shuffles add the
// four rows of the wave, LDS the waves.
__device__ __forceinline__ void table_quad_store(u32 j, const QuadAcc &q, u64 *row) {
    __shared__ u64 sm[NWAVES][12];
    u64 v[4] = {fp::canon(q.g), fp::canon(q.q0), fp::canon(q.q1), fp::canon(q.q2)};  // (below p + 4)
#pragma unroll
    for (int k = 0; k < 4; k++) {
        v[k] = add(v[k], dpp64<0x114, 0xf>(v[k]));  // row_shr:4
        v[k] = add(v[k], dpp64<0x118, 0xf>(v[k]));  // row_shr:8
        v[k] = add(v[k], xor64(v[k], 16));
        v[k] = add(v[k], xor64(v[k], 32));
    }
    const u32 lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane >= 12 && lane < 15) {
#pragma unroll
        for (int k = 0; k < 4; k++) sm[wid][3 * k + (lane - 12)] = v[k];
    }
    (void)j;
    __syncthreads();
    if (threadIdx.x < 12) {
        u64 t = sm[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < NWAVES; w++) t = add(t, sm[w][threadIdx.x]);
        row[threadIdx.x] = t;
    }
}

// Level-0 entries from a wire's sums (phase 2: ADD gates w (v1 + G(t)),
// MUL gates w v1 G(t)).
__device__ __forceinline__ void level0(u32 ph, u64 v1, u64 sA, u64 sC, u64 &A, u64 &C) {
    if (ph == 2) {
        A = add(sA, mul(v1, sC));
        C = mul(v1, sA);
    } else {
        A = sA;
        C = sC;
    }
}

// Level-0 tables of an omega phase and round 0; a thread takes a pair of
// wires.  wire(x, sA, sC) gives the sums of wire x's gates.  GK, PH: the
// gate mix and phase when known at compile time (-1, 0: ph and hasC).
template <int GK, int PH, typename Wire>
__device__ __forceinline__ void level0_round(u32 ph_rt, u32 hasC_rt, u64 npairs, const u64 *F, u64 *At, u64 *Ct,
                                             const ProofPtrs &pp, const Ctx &c, u64 *row, Wire wire) {
    const u32 ph = PH > 0 ? (u32)PH : ph_rt;
    const bool hasC = GK >= 0 ? GK != 1 : hasC_rt != 0;
    const u64 v1 = ph == 2 ? pp.state[1] : 0;
    u64 acc[3] = {0, 0, 0};
    for (u64 m = c.gtid; m < npairs; m += c.gstride) {
        u64 A[2], C[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            u64 sA, sC;
            wire(2 * m + h, sA, sC);
            if (GK == 1 && ph == 2) {  // MUL gates only: sA is zero
                A[h] = mul(v1, sC);
                C[h] = 0;
            } else {
                level0(ph, v1, sA, sC, A[h], C[h]);
            }
            if (!hasC) C[h] = 0;
        }
        st2(At, 2 * m, A[0], A[1]);
        if (hasC) st2(Ct, 2 * m, C[0], C[1]);
        const u64x2 f = ld2(F, 2 * m);
        if (GK == 1)
            table_terms<0>(A[0], A[1], C[0], C[1], f.x, f.y, acc);
        else
            table_terms(A[0], A[1], C[0], C[1], f.x, f.y, acc);
    }
    block_store<3>(acc, row);
}

// Round 0 from the chunk sums: wire x's sums add its chunks
// [xch[x], xch[x+1]).  A lane adds the chunks of its own wire when they are
// few; a wire with more (the pattern entries of pattern matching feed up to
// 2^18 gates) is summed by the whole wave, lanes striding over its chunks,
// one such wire after another.  Whole waves iterate together, so the wave
// reductions see every lane.
constexpr u32 WT0_LANE_CHUNKS = 64;
__device__ __forceinline__ void step_wt0(const Wt0Args &a, const ProofPtrs &pp, const Ctx &c, u64 *row) {
    const u64 v1 = a.ph == 2 ? pp.state[1] : 0;
    const u32 lane = threadIdx.x & 63;
    u64 acc[3] = {0, 0, 0};
    for (u64 base = c.gtid - lane; base < a.npairs; base += c.gstride) {  // wave-uniform
        const u64 m = base + lane;
        const bool on = m < a.npairs;
        u64 A[2], C[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            u32 c0 = 0, c1 = 0;
            if (on) {
                c0 = a.xch[2 * m + h];
                c1 = a.xch[2 * m + h + 1];
            }
            const bool many = c1 - c0 > WT0_LANE_CHUNKS;
            u64 sA = 0, sC = 0;
            if (!many) {
                for (u32 ch = c0; ch < c1; ch++) {
                    sA = add(sA, a.partA[ch]);
                    sC = add(sC, a.partC[ch]);
                }
            }
            for (u64 hm = __ballot(many); hm; hm &= hm - 1) {
                const u32 l = (u32)__ffsll((long long)hm) - 1;  // uniform
                const u32 b0 = (u32)__builtin_amdgcn_readlane((int)c0, l);
                const u32 b1 = (u32)__builtin_amdgcn_readlane((int)c1, l);
                u64 wA = 0, wC = 0;
#pragma unroll 4
                for (u32 ch = b0 + lane; ch < b1; ch += 64) {
                    wA = add(wA, a.partA[ch]);
                    wC = add(wC, a.partC[ch]);
                }
                wA = lane_value(wave_sum63(wA), 63);
                wC = lane_value(wave_sum63(wC), 63);
                if (lane == l) {
                    sA = wA;
                    sC = wC;
                }
            }
            level0(a.ph, v1, sA, sC, A[h], C[h]);
            if (!a.hasC) C[h] = 0;
        }
        if (on) {
            st2(a.A, 2 * m, A[0], A[1]);
            if (a.hasC) st2(a.C, 2 * m, C[0], C[1]);
            const u64x2 f = ld2(a.F, 2 * m);
            table_terms(A[0], A[1], C[0], C[1], f.x, f.y, acc);
        }
    }
    block_store<3>(acc, row);
}

// GK, PH: the gate mix and phase, compile-time (one kernel each) or -1, 0.
template <int GK, int PH>
__device__ __forceinline__ void step_wa0(const Wa0Args &a, const ProofPtrs &pp, const Ctx &c, u64 *row) {
    level0_round<GK, PH>(a.ph, a.hasC, a.npairs, a.Vn, a.A, a.C, pp, c, row, [&](u64 x, u64 &sA, u64 &sC) {
        wire_sums<GK, PH>(a, a.rowptr[x], a.rowptr[x + 1], sA, sC);
    });
}

// HC: whether the layer has a C table, compile-time (one kernel each) or -1.
template <int HC>
__device__ __forceinline__ void step_wt(const WtArgs &a, const Ctx &c, u64 *row) {
    const bool hasC = HC >= 0 ? HC != 0 : a.hasC != 0;
    const u64 r0 = c.r, r1 = c.r2, r01 = mul(r0, r1);
    QuadAcc acc;
    const u32 pend = a.pend;
    auto foldp = [&](const u64 *X, u64 g) {  // level-(k+pend) entry g from level k
        if (pend == 1) {
            const u64x2 p = ld2(X, 2 * g);
            return fold1(p.x, p.y, r0);
        }
        const u64x2 p = ld2(X, 4 * g), q = ld2(X, 4 * g + 2);
        return fold2(p.x, p.y, q.x, q.y, r0, r1, r01);
    };
    // lane g = entry 4u + j of level k+pend (the stride is a multiple of 4)
    for (u64 g = c.gtid; (g >> 2) < a.nu; g += c.gstride) {
        const u32 j = (u32)(g & 3);
        const u64 A = foldp(a.A, g), F = foldp(a.F, g);
        const u64 C = hasC ? foldp(a.C, g) : 0;
        a.An[g] = A;
        a.Fn[g] = F;
        if (hasC) a.Cn[g] = C;
        table_quad<HC>(j, A, C, F, hasC, acc);
    }
    table_quad_store((u32)(c.gtid & 3), acc, row);
}

// ------------------------------------------------------------------ tails
//
// A tail runs the last rounds of a phase in one workgroup, over tables in
// LDS laid out as binary trees: with n = 2^L entries in level 0, level k
// (n_k = n >> k entries) sits at [2n - 2 n_k, 2n - n_k), so pair m of
// level k is the tail's pair q = n - n_k + m, it holds entries 2q, 2q + 1
// and it folds into entry n + q.  Every round first sums its message over
// the level's pairs into partial sums in LDS; a barrier completes them, and
// only after it is the round's challenge used (folds, the p-phase's beta
// prefix); a second barrier publishes the next level.  While a level has at
// least 128 entries every thread takes one pair of every table, adds its
// three terms into 64-pair chunk sums and then folds the pair it holds;
// below that wave t sums value t of the message and then folds table t.
// The partial sums of all rounds are added into the messages at the end.

constexpr int TAIL_TAB = 2 * TAIL_LIM;              // LDS entries per table: all levels
constexpr int TAIL_LOG = 10;                        // log2(TAIL_LIM): rounds of a tail
constexpr int TAIL_CHUNKS = TAIL_LIM / 64;          // 64-pair chunks of a tail
constexpr int TAIL_SLOTS = TAIL_CHUNKS + TAIL_LOG;  // chunk sums, then the small rounds' sums
static_assert((1 << TAIL_LOG) == TAIL_LIM, "TAIL_LOG");
static_assert(TAIL_LIM / 2 <= SBLOCK, "a wide round gives every pair a thread");
static_assert(NWAVES >= 3, "one wave per message value");

__device__ __forceinline__ u64 *tail_lds() {
    __shared__ __align__(16) u64 t[3 * TAIL_TAB];
    return t;
}

// Partial message sums of a tail, per value t: chunk c's sum in slot c
// (rounds of at least 64 pairs), round k's sum in slot TAIL_CHUNKS + k
// (rounds of fewer).
__device__ __forceinline__ u64 (*tail_parts())[TAIL_SLOTS] {
    __shared__ u64 p[3][TAIL_SLOTS];
    return p;
}


// Sum over the wave of field elements, left in lane 63: as wave_sum63, but
// the first three and the last three steps add without reducing (eight
// values below p stay below 2^64), with one reduction after each three.
__device__ __forceinline__ u64 wave_sum63_lazy(u64 v) {
    v += dpp64<0x111, 0xf>(v);  // row_shr:1
    v += dpp64<0x112, 0xf>(v);  // row_shr:2
    v += dpp64<0x114, 0xf>(v);  // row_shr:4
    v = fp::canon(fp::fold64(v));
    v += dpp64<0x118, 0xf>(v);  // row_shr:8
    v += dpp64<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v += dpp64<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    return fp::canon(fp::fold64(v));
}

// A wave's three message terms of one 64-pair chunk c, summed into the
// chunk's partial sums.
__device__ __forceinline__ void chunk_sums(u64 (&t)[3], u32 c, u32 lane) {
    u64 (*mp)[TAIL_SLOTS] = tail_parts();
#pragma unroll
    for (int i = 0; i < 3; i++) t[i] = wave_sum63_lazy(t[i]);
    if (lane == 63) {
#pragma unroll
        for (int i = 0; i < 3; i++) mp[i][c] = t[i];
    }
}

// Value t of round k's message sum from the partials.
__device__ __forceinline__ u64 tail_sum(u32 n, u32 k, u32 t) {
    const u64 (*mp)[TAIL_SLOTS] = tail_parts();
    const u32 half = n >> (k + 1);
    if (half < 64) return mp[t][TAIL_CHUNKS + k];
    u64 s = 0;
    for (u32 c = (n - 2 * half) >> 6; c < (n - half) >> 6; c++) s = add(s, mp[t][c]);
    return s;
}

// X at t = T on the line through (0, x0), (1, x1).
template <int T>
__device__ __forceinline__ u64 line_at(u64 x0, u64 x1) {
    return T == 0 ? x0 : (T == 1 ? x1 : sub(add(x1, x1), x0));
}

// The three terms of one pair of a tail round, canonical: A(t) F(t) (+ C(t))
// at t = 0, 1, 2, the values at t = 2 unreduced (below 3p) in one 128-bit
// sum reduced once.
template <int HC>
__device__ __forceinline__ void tail_pair_terms(u64 A0, u64 A1, u64 C0, u64 C1, u64 F0, u64 F1, u64 (&t)[3]) {
    u128 t0 = fp::wide(A0, F0), t1 = fp::wide(A1, F1);
    u128 t2 = fp::wide(2 * A1 + (fp::P - A0), 2 * F1 + (fp::P - F0));
    if (HC != 0) {
        t0 += C0;
        t1 += C1;
        t2 += 2 * C1 + (fp::P - C0);
    }
    t[0] = fp::red128(t0);
    t[1] = fp::red128(t1);
    t[2] = fp::red128(t2);
}

// Entry e of the level a tail starts from, folded from memory by the
// pending challenge(s) of the prologue.
__device__ __forceinline__ u64 tail_entry(const u64 *X, u32 e, u32 pend, const Ctx &c) {
    if (pend == 0) return X[e];
    if (pend == 1) {
        const u64x2 p = ld2(X, 2 * e);
        return fold1(p.x, p.y, c.r);
    }
    const u64x2 p = ld2(X, 4 * e), q = ld2(X, 4 * e + 2);
    return fold2(p.x, p.y, q.x, q.y, c.r, c.r2, mul(c.r, c.r2));
}

// RNG state of the tail's first round: the prologue drew the pending
// challenges and left the state after them; a tail without them reads it.
__device__ __forceinline__ u64 tail_state(const ProofPtrs &pp, u32 c0, u32 drew, u64 st) {
    __shared__ u64 s_st;
    if (drew) return uniform(st);
    if (threadIdx.x == 0) s_st = pp.rngst[c0];
    __syncthreads();
    return uniform(s_st);
}

// The rounds of an omega tail over tables A, C, F in LDS (level 0 of each,
// n entries, at the start of its area of TAIL_TAB entries): messages to
// msgp, challenges c0, c0 + 1, ... recorded with the RNG states after them
// (and into rec[k], in LDS, when rec is not NULL); F's last entry is v1
// (last = 1) or v2.  Round k's message is, at t = 0, 1, 2, the sum over its
// pairs of A_t F_t + C_t with X_t the line through the pair.  Returns the
// RNG state after the last round.
// HC: whether the phase has a C table, compile-time (1, 0) or -1 to take hc_rt.
template <int HC = -1>
__device__ __forceinline__ u64 wtail_rounds(u64 *A, u64 *Ct, u64 *F, u32 n, bool hc_rt, u64 st, u64 *msgp, u32 c0,
                                            u32 last, u64 *vout, const ProofPtrs &pp, u64 *rec = nullptr) {
    const bool hc = HC >= 0 ? HC != 0 : hc_rt;
    const u32 tid = threadIdx.x, lane = tid & 63;
    const u32 w = (u32)__builtin_amdgcn_readfirstlane((int)(tid >> 6));  // wave-uniform
    const u32 L = 31 - (u32)__builtin_clz(n);
    u64 (*mp)[TAIL_SLOTS] = tail_parts();
    for (u32 k = 0, nk = n; nk > 1; nk >>= 1, k++) {
        const u32 half = nk >> 1, qb = n - nk;
        const u64 r = fp::sm_field(st);  // challenge k: used after message k's sums
        if (half >= 64) {  // thread tid takes pair qb + tid (whole waves)
            const u32 q = qb + tid;
            u64x2 pa = {0, 0}, pc = {0, 0}, pf = {0, 0};
            if (tid < half) {
                pa = ld2(A, 2 * q);
                pf = ld2(F, 2 * q);
                if (hc) pc = ld2(Ct, 2 * q);
                u64 t[3];
                tail_pair_terms<HC == 0 ? 0 : 1>(pa.x, pa.y, pc.x, pc.y, pf.x, pf.y, t);
                chunk_sums(t, q >> 6, lane);
            }
            __syncthreads();  // message k's sums are complete
            if (tid < half) {
                A[n + q] = fold1(pa.x, pa.y, r);
                F[n + q] = fold1(pf.x, pf.y, r);
                if (hc) Ct[n + q] = fold1(pc.x, pc.y, r);
            }
        } else {  // wave t < 3 sums value t over the pairs, lane m < half taking pair qb + m
            const u32 q = qb + lane;
            const bool on = lane < half;
            u64x2 own = {0, 0};
            if (w < 3) {
                u64x2 pa = {0, 0}, pc = {0, 0}, pf = {0, 0};
                if (on) {
                    pa = ld2(A, 2 * q);
                    pf = ld2(F, 2 * q);
                    if (hc) pc = ld2(Ct, 2 * q);
                }
                // value w's term; the values at t = 2 unreduced (below 3p), reduced once
                const u64 xa = w == 0 ? pa.x : (w == 1 ? pa.y : 2 * pa.y + (fp::P - pa.x));
                const u64 xf = w == 0 ? pf.x : (w == 1 ? pf.y : 2 * pf.y + (fp::P - pf.x));
                u128 tw = fp::wide(xa, xf);
                if (HC != 0) tw += w == 0 ? pc.x : (w == 1 ? pc.y : 2 * pc.y + (fp::P - pc.x));
                const u64 term = fp::red128(tw);
                own = w == 0 ? pa : (w == 1 ? pc : pf);
                const u64 v = wave_sum63_lazy(term);
                if (lane == 63) mp[w][TAIL_CHUNKS + k] = v;
            }
            __syncthreads();  // message k's sums are complete
            if (w < 3 && (w != 1 || hc) && on) (w == 0 ? A : (w == 1 ? Ct : F))[n + q] = fold1(own.x, own.y, r);
        }
        if (tid == 0) {
            pp.chals[c0 + k] = r;
            pp.rngst[c0 + k + 1] = st;
            if (rec) rec[k] = r;
        }
        __syncthreads();  // level k + 1 is complete
    }
    if (tid < 3 * L) {
        const u32 k = tid / 3, t = tid - 3 * k;
        msgp[3 * k + t] = tail_sum(n, k, t);
    }
    if (tid == 0) {
        const u64 v = F[2 * n - 2];  // the root
        *vout = v;
        if (last == 1) pp.state[1] = v;
    }
    return st;
}

// HC: whether the phase has a C table, compile-time (one kernel each) or -1.
template <int HC>
__device__ __forceinline__ void step_wtail(const WtailArgs &a, const ProofPtrs &pp, const Ctx c, u32 drew, u64 st0) {
    u64 *tab = tail_lds();
    const u32 tid = threadIdx.x;
    const bool hc = HC >= 0 ? HC != 0 : a.hasC != 0;
    const u32 n = 1u << (a.sp - a.k0);  // entries of level k0, at most TAIL_LIM
    for (u32 e = tid; e < n; e += SBLOCK) {
        const bool on = e < a.live;  // (the grid steps wrote level k0 - pend below live << pend)
        tab[e] = on ? tail_entry(a.A, e, a.pend, c) : 0;
        if (hc) tab[TAIL_TAB + e] = on ? tail_entry(a.C, e, a.pend, c) : 0;
        tab[2 * TAIL_TAB + e] = on ? tail_entry(a.F, e, a.pend, c) : 0;
    }
    const u64 st = tail_state(pp, a.c0, drew, st0);
    __syncthreads();
    wtail_rounds<HC>(tab, tab + TAIL_TAB, tab + 2 * TAIL_TAB, n, hc, st, a.msg, a.c0, a.last, a.vout, pp);
}

// A whole omega phase of a small layer in one workgroup: the eq table of
// the phase's point (a* in phase 1, b* in phase 2) into the workspace, the
// level-0 tables from the wiring (as ST_WA0 forms them) into LDS, then
// every round as a tail.
__device__ __forceinline__ void step_wsmall(const WsmallArgs &a, const ProofPtrs &pp, const Ctx c) {
    u64 *tab = tail_lds();
    const u32 tid = threadIdx.x;
    {
        const u64 *pt = pp.chals + a.eqbase;
        const u64 nlo = 1ull << a.eqL, nhi = 1ull << (a.eqn - a.eqL);
        const u64 beta = pp.state[0];  // phase 1: a*'s lo half carries beta(z, a*)
        for (u64 x = tid; x < nlo + nhi; x += SBLOCK) {
            if (x < nlo)
                a.eqlo[x] = a.w.ph == 1 ? mul(beta, chi_bits(x, pt, a.eqL)) : chi_bits(x, pt, a.eqL);
            else
                a.eqhi[x - nlo] = chi_bits(x - nlo, pt + a.eqL, a.eqn - a.eqL);
        }
    }
    __syncthreads();  // the eq table is read back by this workgroup
    const Wa0Args &w = a.w;
    const bool hc = w.hasC != 0;
    const u64 v1 = w.ph == 2 ? pp.state[1] : 0;
    const u32 n = 1u << a.sp;
    for (u32 x = tid; x < n; x += SBLOCK) {
        u64 sA, sC, A, C;
        wire_sums(w, w.rowptr[x], w.rowptr[x + 1], sA, sC);
        level0(w.ph, v1, sA, sC, A, C);
        tab[x] = A;
        if (hc) tab[TAIL_TAB + x] = C;
        tab[2 * TAIL_TAB + x] = w.Vn[x];
    }
    const u64 st = tail_state(pp, a.c0, 0, 0);
    __syncthreads();
    wtail_rounds(tab, tab + TAIL_TAB, tab + 2 * TAIL_TAB, n, hc, st, a.msg, a.c0, a.last, a.vout, pp);
    (void)c;
}

// p-phase rounds in one workgroup.  B is the table of sums of the eq
// weights of the a-coordinates not yet reached (beta over z's suffix); pair
// m of V goes with B[m].  Round j's message is G(t) = C_j eq_t(z_j) S_t with
// S_t = sum_m B[m] V_t over the pairs and eq_t(z) the line through
// (0, 1 - z), (1, z): 1 - z, z, 3z - 1 at t = 0, 1, 2; C_{j+1} =
// C_j eq(z_j, r_j).  V is a tree as the omega tables; B's level k sits at
// the indexes q of the pairs it goes with, its entry q' of level k+1 being
// the sum of entries 2q' - n and 2q' - n + 1.
//
// ptail_rounds: the rounds over V (level 0: n = 2^L entries) and B (the
// weights of its pairs, level 0: n / 2 entries), both in LDS as trees of
// TAIL_TAB entries.  Lane l holds z_l of the tail's rounds in zr; C is the
// beta prefix before round 0.  Messages go to msg, challenges c0, c0 + 1, ...
// are recorded with the RNG states after them (and into rec[k], in LDS, when
// rec is not NULL).  Returns beta over every round; st becomes the state
// after the last challenge.
__device__ __forceinline__ u64 ptail_rounds(u64 *V, u64 *B, u32 L, u64 zr, u64 C, u64 &st, u32 c0, u64 *msg,
                                            const ProofPtrs &pp, u64 *rec = nullptr) {
    __shared__ u64 s_cz[2][TAIL_LOG];  // C_j and z_j of each round
    const u32 tid = threadIdx.x, lane = tid & 63;
    const u32 w = (u32)__builtin_amdgcn_readfirstlane((int)(tid >> 6));  // wave-uniform
    const u32 n = 1u << L;
    u64 (*mp)[TAIL_SLOTS] = tail_parts();
    for (u32 k = 0, nk = n; nk > 1; nk >>= 1, k++) {
        const u32 half = nk >> 1, qb = n - nk;
        const u64 r = fp::sm_field(st);  // challenge k: used after message k's sums
        const u64 z = lane_value(zr, k);
        if (tid == 0) {
            s_cz[0][k] = C;
            s_cz[1][k] = z;
        }
        if (half >= 64) {  // thread tid takes pair qb + tid (whole waves)
            const u32 q = qb + tid;
            u64x2 pv = {0, 0};
            if (tid < half) {
                pv = ld2(V, 2 * q);
                const u64 b = B[q];
                u64 t[3] = {mul(b, pv.x), mul(b, pv.y), fp::red128(fp::wide(b, 2 * pv.y + (fp::P - pv.x)))};
                chunk_sums(t, q >> 6, lane);
                if (tid < half / 2) {  // B at the pairs of the next level
                    const u32 q2 = n - half + tid;
                    const u64x2 pb = ld2(B, 2 * q2 - n);
                    B[q2] = add(pb.x, pb.y);
                }
            }
            __syncthreads();  // message k's sums are complete
            if (tid < half) V[n + q] = fold1(pv.x, pv.y, r);
        } else {  // wave t < 3 sums value t over the pairs, lane m < half taking pair qb + m
            const u32 q = qb + lane;
            const bool on = lane < half;
            u64x2 pv = {0, 0};
            if (w < 3) {
                u64 b = 0;
                if (on) {
                    pv = ld2(V, 2 * q);
                    b = B[q];
                }
                const u64 x = w == 0 ? pv.x : (w == 1 ? pv.y : 2 * pv.y + (fp::P - pv.x));  // (t = 2: below 3p)
                const u64 v = wave_sum63_lazy(fp::red128(fp::wide(b, x)));
                if (lane == 63) mp[w][TAIL_CHUNKS + k] = v;
                if (w == 1 && lane < half / 2) {  // B at the pairs of the next level
                    const u32 q2 = n - half + lane;
                    const u64x2 pb = ld2(B, 2 * q2 - n);
                    B[q2] = add(pb.x, pb.y);
                }
            }
            __syncthreads();  // message k's sums are complete
            if (w == 0 && on) V[n + q] = fold1(pv.x, pv.y, r);
        }
        C = mul(C, fp::eq(z, r));  // the beta prefix of round k + 1
        if (tid == 0) {
            pp.chals[c0 + k] = r;
            pp.rngst[c0 + k + 1] = st;
            if (rec) rec[k] = r;
        }
        __syncthreads();  // level k + 1 is complete
    }
    if (tid < 3 * L) {
        const u32 k = tid / 3, t = tid - 3 * k;
        const u64 z = s_cz[1][k];
        const u64 e = t == 0 ? sub(1, z) : (t == 1 ? z : sub(add(add(z, z), z), 1));
        msg[3 * k + t] = mul(mul(s_cz[0][k], e), tail_sum(n, k, t));
    }
    return C;
}

// B_0[m] = prod_{k=1}^{s-1} eq(bit k-1 of m, z_k) for m < 2^{s-1}, the
// weights of z's suffix (the p-phase's first round pairs V entries 2m,
// 2m+1); lane l holds z_l in zr.
// The s - 1 factors are multiplied as a balanced tree (a chain of at most
// four products instead of s - 1); tree levels no factor reaches are
// skipped.
__device__ __forceinline__ void suffix_weights(u64 *B, u32 s, u64 zr) {
    const u32 nf = s ? s - 1 : 0;
    for (u32 m = threadIdx.x; m < (1u << s) / 2; m += SBLOCK) {
        u64 f[TAIL_LOG];
#pragma unroll
        for (u32 k = 0; k < TAIL_LOG; k++) f[k] = k < nf ? fp::eqbit((m >> k) & 1, lane_value(zr, k + 1)) : 1;
#pragma unroll
        for (u32 w = 1; w < TAIL_LOG; w *= 2) {
            if (w < nf) {  // (uniform)
#pragma unroll
                for (u32 k = 0; k + w < TAIL_LOG; k += 2 * w) f[k] = mul(f[k], f[k + w]);
            }
        }
        B[m] = f[0];
    }
}

// Remaining p-phase rounds j0..s-1 (ST_PTAIL).  The prologue drew the
// pending challenge(s) up to r_{j0-1} and its finish of round j0-1 computed
// the beta prefix C.
__device__ __forceinline__ void step_ptail(const PtailArgs &a, const ProofPtrs &pp, const Ctx c, u32 drew, u64 st0,
                                           u32 have_c, u64 C0) {
    __shared__ u64 s_c;
    u64 *tab = tail_lds();
    u64 *V = tab, *B = tab + TAIL_TAB;
    const u32 tid = threadIdx.x, lane = tid & 63;
    const u32 L = a.s - a.j0, n = 1u << L;  // entries of V^(j0), at most TAIL_LIM
    for (u32 e = tid; e < n; e += SBLOCK) V[e] = e < a.live ? tail_entry(a.V, e, a.pend, c) : 0;
    const u64 zr = lane < L ? pp.zbuf[a.j0 + lane] : 0;  // z_{j0 + l} in lane l
    if (a.B) {
        for (u32 m = tid; m < n / 2; m += SBLOCK) {  // B_{j0}[m] = B_{j0-1}[2m] + B_{j0-1}[2m+1]
            const u64x2 pb = ld2(a.B, 2 * m);
            B[m] = add(pb.x, pb.y);
        }
    } else {
        suffix_weights(B, L, zr);  // B_{j0}[m] = prod_{k >= 1} eq(bit k-1 of m, z_{j0+k})
    }
    if (!have_c && tid == 0) s_c = pp.state[0];
    u64 st = tail_state(pp, a.c0, drew, st0);
    __syncthreads();
    const u64 C = ptail_rounds(V, B, L, zr, uniform(have_c ? C0 : s_c), st, a.c0, a.msg, pp);
    if (tid == 0) pp.state[0] = C;  // beta(z, a*)
}

// ---------------------------------------------------------- line by folding
//
// h(t) = ~V_{i+1}(l(t)), l(t) = b* + t (c* - b*), is a polynomial of degree
// s' in t.  Folding V along the line coordinate by coordinate (bit k of the
// index, LSB first) turns each entry pair into a polynomial one degree
// higher: with D = P1 - P0 and d_k = c_k - b_k, the fold is
// P0(t) + (b_k + t d_k) D(t), whose coefficient j is P0_j + b_k D_j +
// d_k D_{j-1}.  After all s' folds the one polynomial left is h.  About four
// products an entry, against one per entry and line point for the sums over
// eq tables (ST_LT, ST_LINE), so wide layers take this path.  A thread folds
// 2^tb entries in registers (tb coordinates, 1 <= tb <= 5); the workgroup's 512
// polynomials of degree tb take 9 more coordinates in LDS, one coefficient
// per work item, leaving Q_g of degree D = tb + 9 for the workgroup's block
// g of 2^D entries.  Since h(t) = sum_g Q_g(t) prod_{k >= D} (g_{k-D} ?
// l_k(t) : 1 - l_k(t)), the workgroup then evaluates its term at t = 2..s'
// and writes it as a row (two rows: 16 values a row); ST_FINISH adds the
// rows up.
constexpr u32 LF_LDS = 9;  // coordinates folded in LDS (SBLOCK = 2^9 polynomials)
static_assert((1 << LF_LDS) == SBLOCK, "a workgroup's threads hold 2^9 polynomials");

// The fold of a and b (degree D, in registers) into o (degree D + 1).
template <int D>
__device__ __forceinline__ void fold_poly(const u64 (&a)[D + 1], const u64 (&b)[D + 1], u64 bk, u64 dk,
                                          u64 (&o)[D + 2]) {
    u64 Dprev = 0;
#pragma unroll
    for (int j = 0; j <= D + 1; j++) {
        const int jj = j <= D ? j : D;  // (in range for the unrolled loads)
        const u64 Dj = j <= D ? diff_lz(b[jj], a[jj]) : 0;  // (< 2p: the sum stays below 2^125)
        const u64 a0 = j <= D ? a[jj] : 0;
        o[j] = fp::red128((u128)a0 + fp::wide(bk, Dj) + fp::wide(dk, Dprev));
        Dprev = Dj;
    }
}

template <int N, int D>
__device__ __forceinline__ void fold_level_reg(const u64 (&p)[N][D + 1], u64 (&q)[N / 2][D + 2], u64 bk, u64 dk) {
#pragma unroll
    for (int m = 0; m < N / 2; m++) fold_poly<D>(p[2 * m], p[2 * m + 1], bk, dk, q[m]);
}

// L fold levels in LDS: M polynomials of degree d at src (d + 1 words each,
// one after another) along coordinates k .. k + L - 1, one work item per
// output coefficient, between src and dst in turn; returns the buffer with
// the M >> L polynomials of degree d + L.  Ends with the workgroup in step.
__device__ __forceinline__ u64 *lds_fold(u64 *src, u64 *dst, u32 M, u32 d, u32 k, u32 L, const u64 *bk,
                                         const u64 *dk) {
    for (u32 l = 0; l < L; l++, d++, M >>= 1, k++) {
        const u32 nc = d + 2, items = (M >> 1) * nc;
        const u64 b = bk[k], dl = dk[k];
        for (u32 it = threadIdx.x; it < items; it += SBLOCK) {
            const u32 m = it / nc, j = it - m * nc;
            const u64 *P0 = src + (2 * m) * (d + 1), *P1 = P0 + (d + 1);
            const u64 a0 = j <= d ? P0[j] : 0;
            const u64 Dj = j <= d ? diff_lz(P1[j], P0[j]) : 0;  // (< 2p: the sum stays below 2^125)
            const u64 Dm = j >= 1 ? diff_lz(P1[j - 1], P0[j - 1]) : 0;
            dst[it] = fp::red128((u128)a0 + fp::wide(b, Dj) + fp::wide(dl, Dm));  // (it = m nc + j)
        }
        __syncthreads();
        u64 *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// Register levels D .. TB-1 of N polynomials of degree D; the one left
// (degree TB) goes to out.
template <int N, int D, int TB>
__device__ __forceinline__ void fold_regs(const u64 (&p)[N][D + 1], const u64 *bk, const u64 *dk, u64 *out) {
    if constexpr (D == TB) {
        static_assert(N == 1, "2^TB entries make one polynomial of degree TB");
#pragma unroll
        for (int j = 0; j <= TB; j++) out[j] = p[0][j];
    } else {
        u64 q[N / 2][D + 2];
        fold_level_reg<N, D>(p, q, bk[D], dk[D]);
        fold_regs<N / 2, D + 1, TB>(q, bk, dk, out);
    }
}

template <int TB>
__device__ __forceinline__ void lfold_body(const LfoldArgs &a, const Ctx &c, i32 draw) {
    constexpr int E = 1 << TB;  // entries a thread folds
    u64 *tab = tail_lds();
    u64 *bk = tab, *dk = tab + 32;
    u64 *buf0 = tab + 64, *buf1 = buf0 + SBLOCK * (TB + 1);  // 512 x (TB+1), then 256 x (TB+2) words
    const u32 tid = threadIdx.x;
    // the thread's entries (loaded before the line's coordinates are read)
    const u64 *src = a.V + ((u64)c.lb << (TB + LF_LDS)) + ((u64)tid << TB);
    u64 x[E][1];
#pragma unroll
    for (int e = 0; e < E; e += 2) {
        const u64x2 v = ld2(src, e);
        x[e][0] = v.x;
        x[e + 1][0] = v.y;
    }
    if (tid < a.sp) {  // (the challenge drawn by this launch's prologue is c.r, not yet in chals)
        const i32 bi = (i32)(a.bbase + tid), ci = (i32)(a.cbase + tid);
        const u64 b = bi == draw ? c.r : a.chals[bi], cc = ci == draw ? c.r : a.chals[ci];
        bk[tid] = b;
        dk[tid] = sub(cc, b);
    }
    __syncthreads();
    fold_regs<E, 0, TB>(x, bk, dk, buf0 + tid * (TB + 1));
    __syncthreads();
    constexpr u32 D = TB + LF_LDS;
    const u64 *h = lds_fold(buf0, buf1, SBLOCK, TB, TB, LF_LDS, bk, dk);  // Q_g, degree D
    // Q_g(t) times the weight of this workgroup's block along the remaining
    // coordinates, prod_{k >= D} (g_{k-D} ? l_k(t) : 1 - l_k(t)), at t = 2..s'
    if (tid + 2 <= a.sp) {
        const u64 t = tid + 2;
        u64 q = h[D];
#pragma unroll
        for (int j = D - 1; j >= 0; j--) q = add(mul(q, t), h[j]);
        for (u32 k = D; k < a.sp; k++) {
            const u64 l = add(bk[k], mul(t, dk[k]));
            q = mul(q, (c.lb >> (k - D)) & 1 ? l : sub(1, l));
        }
        a.rows[((u64)(tid / ROW_STRIDE) * c.nb + c.lb) * ROW_STRIDE + tid % ROW_STRIDE] = q;
    }
}

// draw: the challenge index drawn by the launch's prologue (one round's
// finish at most: FIN_W or none), -1 if none.
__device__ __forceinline__ void step_lfold(const LfoldArgs &a, const Ctx &c, i32 draw) {
    switch (a.tb) {
        case 1: lfold_body<1>(a, c, draw); break;
        case 2: lfold_body<2>(a, c, draw); break;
        case 3: lfold_body<3>(a, c, draw); break;
        case 4: lfold_body<4>(a, c, draw); break;
        default: lfold_body<5>(a, c, draw); break;
    }
}

// ---------------------------------------------------------------- top layers
//
// ST_TOP runs the sum-check of the circuit's first layers in one
// workgroup, one layer after the other, as the tails run a phase: the
// p-phase over V_i, the two omega phases over A, C and F = V_{i+1}, and the
// line through b* and c*.  The tables stay in LDS between layers: the
// omega phases leave V_{i+1} as level 0 of F, which is the next layer's
// V_i, so global memory is read only for each V_{i+1} and the wiring and
// written only for messages, challenges and RNG states.  LDS areas (TAIL_TAB
// entries each): X holds B (p-phase), A (omega phases) and the line's point
// tables; Y holds C and, in its last 128 entries, the eq halves of a* and
// b* while the level-0 tables are formed; Z holds V_i, then F.

// lo[x] = chi_x(pt[0..L)) for x < 2^L and hi[x] = chi_x(pt[L..n)) for
// x < 2^(n-L), L = n / 2, so chi_x(pt) = lo[x mod 2^L] hi[x >> L].
__device__ __forceinline__ void eq_halves_lds(const u64 *pt, u32 n, u64 *lo, u64 *hi) {
    const u32 L = n / 2, nlo = 1u << L, nhi = 1u << (n - L);
    for (u32 x = threadIdx.x; x < nlo + nhi; x += SBLOCK) {
        if (x < nlo)
            lo[x] = chi_bits(x, pt, L);
        else
            hi[x - nlo] = chi_bits(x - nlo, pt + L, n - L);
    }
}

// Level 0 of omega phase ph of a top layer: wire x's gates (one chunk)
// summed as wire_sums sums them, with chi_g(a*) and (phase 2)
// chi_in1(b*) from the eq halves in LDS and phase 1's operand V_{i+1}[in2]
// from F in LDS.
__device__ __forceinline__ void top_level0(const TopLayer &Ld, u32 ph, u64 beta, u64 v1, const u64 *ea, u32 La,
                                           const u64 *eb, u32 Lb, const u64 *F, u64 *A, u64 *C, bool hc) {
    const u32 N = 1u << Ld.sp, q = ph - 1;
    const u32 *rowptr = Ld.rowptr[q], *perm = Ld.perm[q], *oths = Ld.oths[q];
    const u8 *types = Ld.types[q];
    const u32 amask = (1u << La) - 1, bmask = (1u << Lb) - 1;
    const u64 *ea_hi = ea + 32, *eb_hi = eb + 32;
    for (u32 x = threadIdx.x; x < N; x += SBLOCK) {
        u64 sA = 0, sC = 0;
        const u32 p0 = rowptr[x], p1 = rowptr[x + 1];
        for (u32 p = p0; p < p1; p++) {
            const u32 g = perm[p], o = oths[p];
            const bool ismul = Ld.kind == 1 || (Ld.kind == 2 && types[p]);  // MUL, or a MUL gate of a mixed layer
            u64 w = mul(beta, mul(ea[g & amask], ea_hi[g >> La]));
            if (ph == 1) {
                const u64 wy = mul(w, F[o]);
                sA = add(sA, ismul ? wy : w);
                sC = add(sC, ismul ? 0 : wy);
            } else {
                w = mul(w, mul(eb[o & bmask], eb_hi[o >> Lb]));
                sA = add(sA, ismul ? 0 : w);
                sC = add(sC, ismul ? w : 0);
            }
        }
        u64 a, c;
        level0(ph, v1, sA, sC, a, c);
        A[x] = a;
        if (hc) C[x] = c;
    }
}

// The line of a top layer: h(t) = ~V_{i+1}(l(t)) for t = 2..sp, l(t) =
// b* + t (c* - b*), over level 0 of F.  The eq halves of point t go to
// tb + 64 (t - 2) (lo, 32 entries) and 32 past it (hi); wave w sums points
// t - 2 = w, w + NWAVES, ..., each lane adding hi lo V over every 64th
// entry in 128 bits, and lane 63 writes h(t) to out[t - 2].
__device__ __forceinline__ void top_line(u32 sp, const u64 *bst, const u64 *cst, const u64 *F, u64 *tb, u64 *out) {
    const u32 T = sp - 1, Ll = sp / 2, Lh = sp - Ll;
    for (u32 e = threadIdx.x; e < T * 64; e += SBLOCK) {
        const u32 tp = e >> 6, j = e & 63;
        const u64 t = tp + 2;
        const bool lo = j < 32;
        const u32 x = lo ? j : j - 32, nb = lo ? Ll : Lh, base = lo ? 0 : Ll;
        if (x < (1u << nb)) {
            u64 v = 1;
            for (u32 k = 0; k < nb; k++) {
                const u64 b = bst[base + k], c = cst[base + k];
                v = mul(v, fp::eqbit((x >> k) & 1, add(b, mul(t, sub(c, b)))));
            }
            tb[e] = v;
        }
    }
    __syncthreads();
    const u32 lane = threadIdx.x & 63;
    const u32 w = (u32)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const u32 N = 1u << sp, m = (1u << Ll) - 1;
    for (u32 tp = w; tp < T; tp += NWAVES) {
        const u64 *lo = tb + 64 * tp, *hi = lo + 32;
        u128 acc = 0;  // at most 16 products below 2^122
        for (u32 x = lane; x < N; x += 64) acc += fp::wide(hi[x >> Ll], mul(lo[x & m], F[x]));
        const u64 v = wave_sum63(fp::red128(acc));
        if (lane == 63) out[tp] = v;
    }
}

__device__ __forceinline__ void step_top(const TopArgs &a, const ProofPtrs &pp) {
    __shared__ u64 s_r[3 * TAIL_LOG];  // the layer's challenges: a*, then b*, then c*
    __shared__ u64 s_st;
    u64 *tab = tail_lds();
    u64 *X = tab, *Y = tab + TAIL_TAB, *Z = tab + 2 * TAIL_TAB;
    u64 *eqa = Y + TAIL_TAB - 128, *eqb = eqa + 64;  // eq halves: lo in [0, 32), hi in [32, 64)
    const u32 tid = threadIdx.x, lane = tid & 63;
    // Evaluation of the layers, nl - 1 down to 0, each from the one below it
    // in LDS (X and Y in turn; Z is not touched), every table also written
    // to memory as ST_EVAL writes it.
    {
        const TopLayer &Lk = a.L[a.nl - 1];
        u64 *src = X, *dst = Y;
        for (u32 e = tid; e < (1u << Lk.sp); e += SBLOCK) src[e] = Lk.Vn[e];
        __syncthreads();
        for (u32 i = a.nl; i-- > 0;) {
            const TopLayer &Ld = a.L[i];
            for (u32 g = tid; g < (1u << Ld.s); g += SBLOCK) {
                u64 v = 0;
                if (g < Ld.S) {
                    const u64 x = src[Ld.in1[g]], y = src[Ld.in2[g]];
                    const bool ismul = Ld.kind == 1 || (Ld.kind == 2 && Ld.type[g]);
                    v = ismul ? mul(x, y) : add(x, y);
                }
                dst[g] = v;
                Ld.V[g] = v;
            }
            __syncthreads();
            u64 *t = src;
            src = dst;
            dst = t;
        }
        // the start (as ST_START): z_0 from the seed's stream, the outputs
        // (V_0, now in src) into the transcript
        const TopLayer &L0 = a.L[0];
        if (tid == 0) {
            u64 st = fp::sm_state(pp.state[2], fp::PURPOSE_GKR);  // state[2] = seed
            pp.rngst[0] = st;
            for (u32 k = 0; k < L0.s; k++) {
                const u64 z = fp::sm_field(st);
                pp.chals[k] = z;
                pp.zbuf[k] = z;
                pp.rngst[k + 1] = st;
            }
            pp.state[0] = 1;
            pp.state[1] = 0;
        }
        for (u32 g = tid; g < L0.S; g += SBLOCK) pp.msgs[g] = src[g];
        __syncthreads();  // the tables, z_0 and the RNG state are read back below
    }
    // V_0, z_0 and the RNG state of the start
    {
        const TopLayer &L0 = a.L[0];
        for (u32 e = tid; e < (1u << L0.s); e += SBLOCK) Z[e] = a.V0[e];
        if (tid == 0) s_st = pp.rngst[L0.co];
    }
    u64 zr = lane < a.L[0].s ? pp.zbuf[lane] : 0;  // z_l of the layer in lane l
    __syncthreads();
    u64 st = uniform(s_st);
    for (u32 i = 0; i < a.nl; i++) {
        const TopLayer &Ld = a.L[i];
        const u32 s = Ld.s, sp = Ld.sp, n = s + 2 * sp, N = 1u << sp;
        const bool hc = Ld.kind != 1;  // a layer with ADD gates has a C table
        // p-phase over V_i (level 0 of Z), B in X; beta starts at 1
        u64 beta = 1;
        if (s > 0) {
            suffix_weights(X, s, zr);
            __syncthreads();
            beta = ptail_rounds(Z, X, s, zr, 1, st, Ld.co, Ld.msg, pp, s_r);
        }
        __syncthreads();  // the p-phase's reads of Z and of its partial sums are done
        // phase 1: F = V_{i+1} into Z, A and C from the gates on in1
        for (u32 e = tid; e < N; e += SBLOCK) Z[e] = Ld.Vn[e];
        eq_halves_lds(s_r, s, eqa, eqa + 32);
        __syncthreads();
        top_level0(Ld, 1, beta, 0, eqa, s / 2, eqb, 0, Z, X, Y, hc);
        __syncthreads();
        st = wtail_rounds(X, Y, Z, N, hc, st, Ld.msg + 3 * s, Ld.co + s, 1, Ld.msg + 3 * n, pp, s_r + s);
        const u64 v1 = Z[2 * N - 2];  // the root of F
        __syncthreads();  // phase 1's partial sums are read; its tree in Y is no longer needed
        // phase 2: the gates on in2, with v1
        eq_halves_lds(s_r, s, eqa, eqa + 32);
        eq_halves_lds(s_r + s, sp, eqb, eqb + 32);
        __syncthreads();
        top_level0(Ld, 2, beta, v1, eqa, s / 2, eqb, sp / 2, Z, X, Y, hc);
        __syncthreads();
        st = wtail_rounds(X, Y, Z, N, hc, st, Ld.msg + 3 * (s + sp), Ld.co + s + sp, 2, Ld.msg + 3 * n + 1, pp,
                          s_r + s + sp);
        __syncthreads();
        // the line (level 0 of Z is still V_{i+1}); its point tables in X
        if (sp >= 2) {
            top_line(sp, s_r + s, s_r + s + sp, Z, X, Ld.msg + 3 * n + 2);
            __syncthreads();
        }
        // tau and z_{i+1} = l(tau) for the next layer of this step (the
        // step after it draws the last layer's tau)
        if (i + 1 < a.nl) {
            const u64 tau = fp::sm_field(st);
            if (tid == 0) {
                pp.chals[Ld.co + n] = tau;
                pp.rngst[Ld.co + n + 1] = st;
            }
            const u64 b = lane < sp ? s_r[s + lane] : 0, c = lane < sp ? s_r[s + sp + lane] : 0;
            zr = add(b, mul(tau, sub(c, b)));
            __syncthreads();  // s_r is read before the next layer records into it
        }
    }
}

// ---------------------------------------------------------------- kernel

// One step on workgroup lb.  Workgroups [0, nblocks) run the body; a step
// that finishes the previous round has one more workgroup, lb == nblocks,
// which only folds the previous rows into the message (so that work runs
// beside the body instead of ahead of it) and records the drawn challenge.
template <u32 KIND, int GK, int PH>
__device__ __forceinline__ void run_step(const StepDesc &sd, u32 lb) {
    __shared__ u64 s_c;
    __shared__ u64 s_pt[64];  // a point (EQ), or b* and c* (LT), or z_{i+1} (FIN_LINE)
    const Fin &f = sd.fin;
    const ProofPtrs &pp = sd.pp;
    const u32 kind = KIND == KALL ? sd.kind : KIND;
    const bool tail = kind == ST_WTAIL || kind == ST_PTAIL || kind == ST_WSMALL ||
                      kind == ST_TOP;  // one workgroup does everything
    const bool has_fin = f.kind != FIN_NONE;
    const bool split = has_fin && !tail;  // workgroup nblocks finishes, the others run the body
    const bool fin_block = split && lb == sd.nblocks;
    const bool recorder = split ? fin_block : lb == 0;
    Ctx c;
    c.lb = lb;
    c.nb = sd.nblocks;
    c.gtid = (u64)c.lb * SBLOCK + threadIdx.x;
    c.gstride = (u64)c.nb * SBLOCK;

    // --- prologue: the challenge.  Every thread of every workgroup draws the
    // same value from the state in memory (a uniform load), so nothing waits
    // for a barrier before the body's first loads.
    u64 st_after = 0;
    c.r = 0;
    c.r2 = 0;
    if (f.draw >= 0) {
        u64 st = pp.rngst[f.draw];
        c.r = fp::sm_field(st);
        const u64 st1 = st;
        const bool two = f.kind == FIN_P2 || f.kind == FIN_T2;  // two rounds finish here
        if (two) c.r2 = fp::sm_field(st);
        if (recorder && threadIdx.x == 0) {
            pp.chals[f.draw] = c.r;
            pp.rngst[f.draw + 1] = st1;
            if (two) {
                pp.chals[f.draw + 1] = c.r2;
                pp.rngst[f.draw + 2] = st;
            }
        }
        st_after = st;  // the state after the drawn challenge(s)
    }
    TailIn ti = {st_after, 0, f.draw >= 0 ? 1u : 0u, 0u};
    // points assembled in LDS (challenges drawn by earlier launches are in
    // chals; the one drawn just now is c.r)
    const bool line_fin = (fin_mask(KIND) & (1u << FIN_LINE)) && f.kind == FIN_LINE;
    if (line_fin || kind == ST_EQ || kind == ST_LT) {  // (uniform)
        if (line_fin && threadIdx.x < f.sp) {
            const u64 bb = f.bstar[threadIdx.x], cc = f.cstar[threadIdx.x];
            s_pt[threadIdx.x] = add(bb, mul(c.r, sub(cc, bb)));  // z_{i+1} = l(tau)
        }
        if (kind == ST_EQ && sd.u.eq.point == PT_Z && f.kind != FIN_LINE &&
            threadIdx.x < sd.u.eq.base + sd.u.eq.n)
            s_pt[threadIdx.x] = pp.zbuf[threadIdx.x];  // z of the layer, already recorded
        if (kind == ST_EQ && sd.u.eq.point == PT_CHAL && threadIdx.x < sd.u.eq.n) {
            const i32 ci = (i32)(sd.u.eq.base + threadIdx.x);
            s_pt[threadIdx.x] = ci == f.draw ? c.r : pp.chals[ci];
        }
        if (kind == ST_LT && threadIdx.x < 2 * sd.u.lt.sp) {
            const u32 sp = sd.u.lt.sp;
            const i32 ci = (i32)(threadIdx.x < sp ? sd.u.lt.bbase + threadIdx.x
                                                  : sd.u.lt.cbase + threadIdx.x - sp);
            s_pt[threadIdx.x] = ci == f.draw ? c.r : pp.chals[ci];
        }
        __syncthreads();
    }
    if (fin_block || (tail && has_fin)) {
        fin_inline<KIND>(sd, c, s_pt, &s_c);
        if (fin_block) return;
    }
    if (tail && has_fin) {
        if (kind == ST_PTAIL && (f.kind == FIN_P || f.kind == FIN_P2)) {
            __syncthreads();
            ti.have_c = 1;
            ti.C = s_c;
        }
        if ((fin_mask(KIND) & (1u << FIN_LINE)) && f.kind == FIN_LINE) __syncthreads();  // z_{i+1} stored
    }

    // --- body
    u64 *row = sd.rows ? sd.rows + (u64)c.lb * ROW_STRIDE : nullptr;
    switch (kind) {
        case ST_LOAD: step_load(sd.u.load, pp, c); break;
        case ST_EVAL: step_eval(sd.u.eval, c); break;
        case ST_START: step_start(sd.u.start, pp, c); break;
        case ST_EQ:
            step_eq(sd.u.eq, c, sd.u.eq.point == PT_Z ? s_pt + sd.u.eq.base : s_pt, pp);
            break;
        case ST_P: step_p<KIND == ST_P ? GK : -1>(sd.u.p, c, row); break;
        case ST_W: {
            const WArgs &a = sd.u.w;
            if (GK >= 0) {
                step_w<GK < 0 ? 0 : GK, PH < 1 ? 1 : PH>(a, c, pp, row);
            } else if (a.ph == 1) {
                if (a.kind == 0) step_w<0, 1>(a, c, pp, row);
                else if (a.kind == 1) step_w<1, 1>(a, c, pp, row);
                else step_w<2, 1>(a, c, pp, row);
            } else {
                if (a.kind == 0) step_w<0, 2>(a, c, pp, row);
                else if (a.kind == 1) step_w<1, 2>(a, c, pp, row);
                else step_w<2, 2>(a, c, pp, row);
            }
            break;
        }
        case ST_FOLD: step_fold(sd.u.fold, c); break;
        case ST_LT: step_lt(sd.u.lt, c, s_pt, s_pt + sd.u.lt.sp); break;
        case ST_LINE: step_line(sd.u.line, c, row); break;
        case ST_WAGG: step_wagg<KIND == ST_WAGG ? GK : -1, KIND == ST_WAGG ? PH : 0>(sd.u.wagg, pp, c); break;
        case ST_WT0: step_wt0(sd.u.wt0, pp, c, row); break;
        case ST_WA0: step_wa0<KIND == ST_WA0 ? GK : -1, KIND == ST_WA0 ? PH : 0>(sd.u.wa0, pp, c, row); break;
        case ST_WT: step_wt<KIND == ST_WT ? GK : -1>(sd.u.wt, c, row); break;
        case ST_WTAIL: step_wtail<KIND == ST_WTAIL ? GK : -1>(sd.u.wtail, pp, c, ti.drew, ti.st); break;
        case ST_PTAIL: step_ptail(sd.u.ptail, pp, c, ti.drew, ti.st, ti.have_c, ti.C); break;
        case ST_FINISH: step_finish(sd.u.finish, c); break;
        case ST_WSMALL: step_wsmall(sd.u.wsmall, pp, c); break;
        case ST_TOP: step_top(sd.u.top, pp); break;
        case ST_LFOLD: step_lfold(sd.u.lfold, c, f.draw); break;
        case ST_SGE:
            if (c.lb == 0 && threadIdx.x == 0) {
                const u64 v = sd.u.sge.Vn[0];
                sd.u.sge.vslot[0] = v;
                sd.u.sge.vslot[1] = v;
                pp.state[1] = v;
            }
            break;
        default: break;
    }
}

// A single proof's step, its descriptor passed by value as kernel argument;
// one instantiation per step kind (and per gate mix and phase for omega
// rounds) keeps each kernel's code and registers to what the kind needs.
template <u32 KIND, int GK, int PH>
__global__ void __launch_bounds__(SBLOCK) k_step_one(const StepDesc sd) {
    run_step<KIND, GK, PH>(sd, blockIdx.x);
}

// One step of each of several proofs.
__global__ void __launch_bounds__(SBLOCK) k_step_jobs(const JobEntry *__restrict__ jobs, u32 njobs) {
    u32 lo = 0, hi = njobs;
    const u32 b = blockIdx.x;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (jobs[mid].block0 <= b) lo = mid; else hi = mid;
    }
    run_step<KALL, -1, 0>(*jobs[lo].step, b - jobs[lo].block0);
}

// One step of each of several proofs, the job table in the kernel arguments.
__global__ void __launch_bounds__(SBLOCK) k_step_table(const JobTable t) {
    u32 lo = 0, hi = t.n;
    const u32 b = blockIdx.x;
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (t.e[mid].block0 <= b) lo = mid; else hi = mid;
    }
    run_step<KALL, -1, 0>(*t.e[lo].step, b - t.e[lo].block0);
}

hipError_t launch_step_table(hipStream_t st, const JobTable &t) {
    hipLaunchKernelGGL(k_step_table, dim3(t.total), dim3(SBLOCK), 0, st, t);
    return hipGetLastError();
}

u32 step_grid(const StepDesc &sd) {
    if (sd.kind == ST_WTAIL || sd.kind == ST_PTAIL || sd.kind == ST_WSMALL || sd.kind == ST_TOP) return 1;
    return sd.nblocks + (sd.fin.kind != FIN_NONE ? 1 : 0);
}

hipError_t launch_step(hipStream_t st, const StepDesc &sd, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 g(step_grid(sd)), b(SBLOCK);
    // with events: the dispatch itself is timed (hipExtLaunchKernelGGL)
#define L1(K) hipExtLaunchKernelGGL((k_step_one<K, -1, 0>), g, b, 0, st, ev0, ev1, 0, sd)
#define LW(G, PH) hipExtLaunchKernelGGL((k_step_one<ST_W, G, PH>), g, b, 0, st, ev0, ev1, 0, sd)
#define LK(K, G, PH) hipExtLaunchKernelGGL((k_step_one<K, G, PH>), g, b, 0, st, ev0, ev1, 0, sd)
    switch (sd.kind) {
        case ST_LOAD: L1(ST_LOAD); break;
        case ST_EVAL: L1(ST_EVAL); break;
        case ST_START: L1(ST_START); break;
        case ST_EQ: L1(ST_EQ); break;
        case ST_P:  // one kernel for the phase's first step, one for the others
            if (sd.u.p.first) LK(ST_P, 1, 0); else LK(ST_P, 0, 0);
            break;
        case ST_W:
            if (sd.u.w.ph == 1) {
                if (sd.u.w.kind == 0) LW(0, 1); else if (sd.u.w.kind == 1) LW(1, 1); else LW(2, 1);
            } else {
                if (sd.u.w.kind == 0) LW(0, 2); else if (sd.u.w.kind == 1) LW(1, 2); else LW(2, 2);
            }
            break;
        case ST_FOLD: L1(ST_FOLD); break;
        case ST_LT: L1(ST_LT); break;
        case ST_LINE: L1(ST_LINE); break;
        case ST_SGE: L1(ST_SGE); break;
        case ST_WAGG: {  // one kernel per gate mix and phase
            const u32 k = sd.u.wagg.kind, ph = sd.u.wagg.ph;
            if (ph == 1) {
                if (k == 0) LK(ST_WAGG, 0, 1); else if (k == 1) LK(ST_WAGG, 1, 1); else LK(ST_WAGG, 2, 1);
            } else {
                if (k == 0) LK(ST_WAGG, 0, 2); else if (k == 1) LK(ST_WAGG, 1, 2); else LK(ST_WAGG, 2, 2);
            }
            break;
        }
        case ST_WT0: L1(ST_WT0); break;
        case ST_WA0: {  // one kernel per gate mix and phase
            const u32 k = sd.u.wa0.kind, ph = sd.u.wa0.ph;
            if (ph == 1) {
                if (k == 0) LK(ST_WA0, 0, 1); else if (k == 1) LK(ST_WA0, 1, 1); else LK(ST_WA0, 2, 1);
            } else {
                if (k == 0) LK(ST_WA0, 0, 2); else if (k == 1) LK(ST_WA0, 1, 2); else LK(ST_WA0, 2, 2);
            }
            break;
        }
        case ST_WT:  // one kernel with a C table, one without
            if (sd.u.wt.hasC) LK(ST_WT, 1, 0); else LK(ST_WT, 0, 0);
            break;
        case ST_WTAIL:  // one kernel with a C table, one without
            if (sd.u.wtail.hasC) LK(ST_WTAIL, 1, 0); else LK(ST_WTAIL, 0, 0);
            break;
        case ST_PTAIL: L1(ST_PTAIL); break;
        case ST_FINISH: L1(ST_FINISH); break;
        case ST_WSMALL: L1(ST_WSMALL); break;
        case ST_TOP: L1(ST_TOP); break;
        case ST_LFOLD: L1(ST_LFOLD); break;
        default: L1(ST_END); break;
    }
#undef L1
#undef LW
#undef LK
    return hipGetLastError();
}

hipError_t launch_steps(hipStream_t st, const JobEntry *jobs, u32 njobs, u32 total_blocks,
                        hipEvent_t ev0, hipEvent_t ev1) {
    hipExtLaunchKernelGGL(k_step_jobs, dim3(total_blocks), dim3(SBLOCK), 0, st, ev0, ev1, 0, jobs, njobs);
    return hipGetLastError();
}

// ------------------------------------------------------------- batches

// Proof q's seed and input pointer into its state; range flag cleared.
__global__ void k_batch_setup(const BatchSlot *slots, u32 n) {
    const u32 q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) {
        u64 *st = slots[q].state;
        st[2] = slots[q].seed;
        st[3] = slots[q].input;
        st[4] = 0;
    }
}

// Transcripts (and range flags) of the batch into one contiguous buffer:
// proof q's msgs at out[slots[q].out_off ...], its flag at out[slots[q].flag_off].
__global__ void k_batch_gather(const BatchSlot *slots, u32 n, u64 *out) {
    const u32 q = blockIdx.x;
    if (q >= n) return;
    const BatchSlot &s = slots[q];
    for (u64 k = threadIdx.x; k < s.n_msgs; k += blockDim.x) out[s.out_off + k] = s.msgs[k];
    if (threadIdx.x == 0) out[s.flag_off] = s.state[4];
}

hipError_t launch_batch_setup(hipStream_t st, const BatchSlot *slots, u32 n) {
    hipLaunchKernelGGL(k_batch_setup, dim3((n + 255) / 256), dim3(256), 0, st, slots, n);
    return hipGetLastError();
}

hipError_t launch_batch_gather(hipStream_t st, const BatchSlot *slots, u32 n, u64 *out) {
    hipLaunchKernelGGL(k_batch_gather, dim3(n), dim3(256), 0, st, slots, n, out);
    return hipGetLastError();
}

}  // namespace gkr
