// kernels.hip -- HIP kernels (gfx950) of the GKR prover's per-layer
// sum-check over F_p, p = 2^61 - 1, of its verifier, and of the F2
// sum-check.
//
// Sec. 4.1.1: each gate contributes independently to the prover's message;
// a workgroup sums its gates' contributions (wave64 shuffles, then LDS),
// writes one row of partial sums, and a one-workgroup *_final kernel folds
// the rows, writes the message and only then draws the next challenge on
// the device.  All arithmetic is exact modular integer arithmetic (no
// floating point, Sec. 5.1), so any summation order gives identical bits.
#include "fp61.hpp"
#include "kernels.hpp"

namespace gkr {

using fp::add;
using fp::mul;
using fp::P;
using fp::sub;

struct alignas(16) u64x2 {
    u64 x, y;
};

__device__ __forceinline__ u64x2 ld2(const u64 *p, u64 i) {
    return *reinterpret_cast<const u64x2 *>(p + i);
}
__device__ __forceinline__ void st2(u64 *p, u64 i, u64 a, u64 b) {
    u64x2 v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<u64x2 *>(p + i) = v;
}

#define GTID ((u64)blockIdx.x * blockDim.x + threadIdx.x)
#define GSTRIDE ((u64)gridDim.x * blockDim.x)

// ---------------------------------------------------------------- reductions

template <int K>
__device__ __forceinline__ void wave_reduce(u64 (&v)[K]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = add(v[k], __shfl_xor(v[k], o));
    }
}

// Sum v over the workgroup; thread k < K writes total k to out[k].
template <int K>
__device__ __forceinline__ void block_store(u64 (&v)[K], u64 *out) {
    __shared__ u64 sm[K][BLOCK / 64];
    wave_reduce<K>(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) sm[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        u64 a = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; w++) a = add(a, sm[threadIdx.x][w]);
        out[threadIdx.x] = a;
    }
}

// One workgroup: fold nparts rows of K values; totals land in tot[] for
// thread 0 (and every thread, through LDS).
template <int K>
__device__ __forceinline__ void rows_total(int nparts, const u64 *partials, u64 (&tot)[K]) {
    __shared__ u64 res[K];
    u64 v[K];
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = 0;
    for (int r = threadIdx.x; r < nparts; r += BLOCK) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = add(v[k], partials[(u64)r * K + k]);
    }
    block_store<K>(v, res);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) tot[k] = res[k];
}

__device__ __forceinline__ u64 draw(ProofState *ps) {
    u64 s = ps->rng;
    u64 r = fp::sm_field(s);
    ps->rng = s;
    return r;
}

// ----------------------------------------------------------- evaluation (a3)

__global__ void __launch_bounds__(BLOCK) k_load_inputs(const u64 *src, u32 S, u64 npad, u64 *V,
                                                       u32 *bad) {
    u32 flag = 0;
    for (u64 g = GTID; g < npad; g += GSTRIDE) {
        u64 v = 0;
        if (g < S) {
            v = src[g];
            if (v >= P) flag = 1;
        }
        V[g] = v;
    }
    if (flag) atomicOr(bad, 1u);
}

hipError_t launch_load_inputs(hipStream_t st, const u64 *src, u32 S, u64 npad, u64 *V,
                              u32 *bad_flag) {
    hipLaunchKernelGGL(k_load_inputs, dim3(blocks_for(npad, 4)), dim3(BLOCK), 0, st, src, S, npad,
                       V, bad_flag);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_check_range(const u64 *src, u64 n, u32 *bad) {
    u32 flag = 0;
    for (u64 g = GTID; g < n; g += GSTRIDE) flag |= src[g] >= P;
    if (flag) atomicOr(bad, 1u);
}

hipError_t launch_check_range(hipStream_t st, const u64 *src, u64 n, u32 *bad_flag) {
    hipLaunchKernelGGL(k_check_range, dim3(blocks_for(n, 4)), dim3(BLOCK), 0, st, src, n, bad_flag);
    return hipGetLastError();
}

template <int KIND>
__global__ void __launch_bounds__(BLOCK) k_eval(u32 S, u64 npad, const u8 *type, const u32 *in1,
                                                const u32 *in2, const u64 *Vn, u64 *V) {
    for (u64 g = GTID; g < npad; g += GSTRIDE) {
        u64 v = 0;
        if (g < S) {
            u64 x = Vn[in1[g]], y = Vn[in2[g]];
            bool ismul = KIND == KIND_MUL || (KIND == KIND_MIXED && type[g]);
            v = ismul ? mul(x, y) : add(x, y);
        }
        V[g] = v;
    }
}

hipError_t launch_eval(hipStream_t st, int kind, u32 S, u64 npad, const u8 *type, const u32 *in1,
                       const u32 *in2, const u64 *Vn, u64 *V) {
    dim3 g(blocks_for(npad, 4)), b(BLOCK);
    switch (kind) {
        case KIND_ADD: hipLaunchKernelGGL(k_eval<KIND_ADD>, g, b, 0, st, S, npad, type, in1, in2, Vn, V); break;
        case KIND_MUL: hipLaunchKernelGGL(k_eval<KIND_MUL>, g, b, 0, st, S, npad, type, in1, in2, Vn, V); break;
        default: hipLaunchKernelGGL(k_eval<KIND_MIXED>, g, b, 0, st, S, npad, type, in1, in2, Vn, V); break;
    }
    return hipGetLastError();
}

// --------------------------------------------------------- proof bookkeeping

__global__ void __launch_bounds__(BLOCK) k_init_proof(ProofState *ps, u64 seed, u32 s0, const u64 *V0,
                                                      u32 S0, u64 *msgs, u64 *chals, u64 *zbuf) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        u64 s = fp::sm_state(seed, fp::PURPOSE_GKR);
        for (u32 k = 0; k < s0; k++) {
            u64 z = fp::sm_field(s);
            chals[k] = z;
            zbuf[k] = z;
        }
        ps->rng = s;
        ps->betaC = 1;
        ps->v1 = 0;
    }
    for (u64 g = GTID; g < S0; g += GSTRIDE) msgs[g] = V0[g];
}

hipError_t launch_init_proof(hipStream_t st, ProofState *ps, u64 seed, u32 s0, const u64 *V0,
                             u32 S0, u64 *msgs, u64 *chals, u64 *zbuf) {
    hipLaunchKernelGGL(k_init_proof, dim3(blocks_for(S0, 4)), dim3(BLOCK), 0, st, ps, seed, s0, V0,
                       S0, msgs, chals, zbuf);
    return hipGetLastError();
}

// chi over the bits of x of the coordinates pt[0..n)
__device__ __forceinline__ u64 chi_bits(u64 x, const u64 *pt, u32 n) {
    u64 e = 1;
    for (u32 k = 0; k < n; k++) e = mul(e, fp::eqbit((u32)((x >> k) & 1), pt[k]));
    return e;
}

__global__ void __launch_bounds__(BLOCK) k_eq_halves(const u64 *pt, u32 s, u32 L, u64 *lo, u64 *hi) {
    const u64 nlo = 1ull << L, nhi = 1ull << (s - L);
    for (u64 x = GTID; x < nlo + nhi; x += GSTRIDE) {
        if (x < nlo)
            lo[x] = chi_bits(x, pt, L);
        else
            hi[x - nlo] = chi_bits(x - nlo, pt + L, s - L);
    }
}

hipError_t launch_eq_halves(hipStream_t st, const u64 *pt, u32 s, u32 L, u64 *lo, u64 *hi) {
    u64 n = (1ull << L) + (1ull << (s - L));
    hipLaunchKernelGGL(k_eq_halves, dim3(blocks_for(n)), dim3(BLOCK), 0, st, pt, s, L, lo, hi);
    return hipGetLastError();
}

// ------------------------------------------------------- p-phase (a5, a7, a8)

template <bool FIRST>
__global__ void __launch_bounds__(BLOCK) k_pphase(u64 nm, const u64 *Vsrc, u64 *Vout,
                                                  const u64 *Bprev, u64 *Bout, const u64 *zlo,
                                                  const u64 *zhi, u32 L, const u64 *rptr,
                                                  u64 *partials) {
    u64 r = 0;
    if (!FIRST) r = *rptr;
    const u64 mask = (1ull << L) - 1;
    u64 acc[2] = {0, 0};
    for (u64 m = GTID; m < nm; m += GSTRIDE) {
        u64 v0, v1, b;
        if (FIRST) {
            u64x2 p = ld2(Vsrc, 2 * m);
            v0 = p.x;
            v1 = p.y;
            b = mul(zlo[m & mask], zhi[m >> L]);
        } else {
            u64x2 p = ld2(Vsrc, 4 * m), q = ld2(Vsrc, 4 * m + 2);
            v0 = add(p.x, mul(r, sub(p.y, p.x)));
            v1 = add(q.x, mul(r, sub(q.y, q.x)));
            if (Vout) st2(Vout, 2 * m, v0, v1);
            u64x2 bb = ld2(Bprev, 2 * m);
            b = add(bb.x, bb.y);
        }
        if (Bout) Bout[m] = b;
        acc[0] = add(acc[0], mul(b, v0));
        acc[1] = add(acc[1], mul(b, v1));
    }
    block_store<2>(acc, partials + 2 * (u64)blockIdx.x);
}

hipError_t launch_pphase(hipStream_t st, bool first, u64 nm, const u64 *Vsrc, u64 *Vout,
                         const u64 *Bprev, u64 *Bout, const u64 *zlo, const u64 *zhi, u32 L,
                         const u64 *rptr, u64 *partials, int *nblocks) {
    int nb = blocks_for(nm, 2);
    *nblocks = nb;
    if (first)
        hipLaunchKernelGGL(k_pphase<true>, dim3(nb), dim3(BLOCK), 0, st, nm, Vsrc, Vout, Bprev, Bout,
                           zlo, zhi, L, rptr, partials);
    else
        hipLaunchKernelGGL(k_pphase<false>, dim3(nb), dim3(BLOCK), 0, st, nm, Vsrc, Vout, Bprev,
                           Bout, zlo, zhi, L, rptr, partials);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_pfinal(int nparts, const u64 *partials, ProofState *ps,
                                                  const u64 *zj, u64 *msg, u64 *chal) {
    u64 t[2];
    rows_total<2>(nparts, partials, t);
    if (threadIdx.x == 0) {
        const u64 z = *zj, C = ps->betaC, S0 = t[0], S1 = t[1];
        msg[0] = mul(mul(C, sub(1, z)), S0);
        msg[1] = mul(mul(C, z), S1);
        const u64 c3 = sub(add(add(z, z), z), 1);  // eq(z, 2) = 3z - 1
        msg[2] = mul(mul(C, c3), sub(add(S1, S1), S0));
        const u64 r = draw(ps);
        *chal = r;
        ps->betaC = mul(C, fp::eq(z, r));
    }
}

hipError_t launch_pfinal(hipStream_t st, int nparts, const u64 *partials, ProofState *ps,
                         const u64 *zj, u64 *msg, u64 *chal) {
    hipLaunchKernelGGL(k_pfinal, dim3(1), dim3(BLOCK), 0, st, nparts, partials, ps, zj, msg, chal);
    return hipGetLastError();
}

// ------------------------------------------------- omega-phases (a6, a7, a8)
//
// Gate g with bound-wire index idx, at round k of its phase:
//   term_g(t) = w_g eq(bit_k(idx), t) (F(t) + off_g)
// with F(t) = (1-t) F[2m] + t F[2m+1], m = idx >> (k+1), the extension of
// V_{i+1} at the partially bound point.  MUL gates carry their fixed
// operand inside w (off = 0), ADD gates in off.  With P0 = w (F[2m] + off),
// P1 = w (F[2m+1] + off):  bit 0 adds P0 at t=0 and P0 - 2 P1 at t=2;
// bit 1 adds P1 at t=1 and 4 P1 - 2 P0 at t=2.

template <int KIND, int PH, bool INIT, bool WRITE_W>
__global__ void __launch_bounds__(BLOCK) k_omega(OmegaArgs a) {
    u64 r = 0, omr = 0;
    if (!INIT) {
        r = *a.rptr;
        omr = sub(1, r);
    }
    u64 wbase = 0, v1 = 0;
    if (INIT) wbase = a.ps->betaC;  // beta(z, a*) once the a-variables are bound
    if (PH == 2) v1 = a.ps->v1;
    const u64 amask = (1ull << a.La) - 1, bmask = (1ull << a.Lb) - 1;
    const u32 k = a.k;
    u64 acc[4] = {0, 0, 0, 0};
    for (u64 g = GTID; g < a.S; g += GSTRIDE) {
        const u32 idx = a.idx[g];
        const bool ismul = KIND == KIND_MUL || (KIND == KIND_MIXED && a.type[g]);
        u64 wt, of;
        if (INIT) {
            u64 wg = mul(wbase, mul(a.alo[g & amask], a.ahi[g >> a.La]));
            if (PH == 1) {
                const u64 y = a.Vn[a.oth[g]];
                wt = ismul ? mul(wg, y) : wg;
                of = ismul ? 0 : y;
                if (KIND != KIND_MUL) a.off[g] = of;
            } else {
                const u32 i1 = a.oth[g];
                wg = mul(wg, mul(a.blo[i1 & bmask], a.bhi[i1 >> a.Lb]));
                wt = ismul ? mul(wg, v1) : wg;
                of = ismul ? 0 : v1;
            }
        } else {
            wt = mul(a.w[g], ((idx >> (k - 1)) & 1) ? r : omr);
            if (PH == 1)
                of = KIND == KIND_MUL ? 0 : a.off[g];
            else
                of = ismul ? 0 : v1;
        }
        const u64x2 f = ld2(a.F, ((u64)idx >> (k + 1)) << 1);
        const u64 P0 = mul(wt, add(f.x, of)), P1 = mul(wt, add(f.y, of));
        if ((idx >> k) & 1) {
            acc[2] = add(acc[2], P0);
            acc[3] = add(acc[3], P1);
        } else {
            acc[0] = add(acc[0], P0);
            acc[1] = add(acc[1], P1);
        }
        if (WRITE_W) a.w[g] = wt;
    }
    block_store<4>(acc, a.partials + 4 * (u64)blockIdx.x);
}

template <int KIND, int PH>
static void launch_omega_k(hipStream_t st, const OmegaArgs &a, int nb) {
    dim3 g(nb), b(BLOCK);
    if (a.init) {
        if (a.write_w)
            hipLaunchKernelGGL((k_omega<KIND, PH, true, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((k_omega<KIND, PH, true, false>), g, b, 0, st, a);
    } else {
        if (a.write_w)
            hipLaunchKernelGGL((k_omega<KIND, PH, false, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((k_omega<KIND, PH, false, false>), g, b, 0, st, a);
    }
}

hipError_t launch_omega(hipStream_t st, const OmegaArgs &a, int *nblocks) {
    int nb = blocks_for(a.S, 4);
    *nblocks = nb;
    if (a.ph == 1) {
        if (a.kind == KIND_ADD) launch_omega_k<KIND_ADD, 1>(st, a, nb);
        else if (a.kind == KIND_MUL) launch_omega_k<KIND_MUL, 1>(st, a, nb);
        else launch_omega_k<KIND_MIXED, 1>(st, a, nb);
    } else {
        if (a.kind == KIND_ADD) launch_omega_k<KIND_ADD, 2>(st, a, nb);
        else if (a.kind == KIND_MUL) launch_omega_k<KIND_MUL, 2>(st, a, nb);
        else launch_omega_k<KIND_MIXED, 2>(st, a, nb);
    }
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_wfinal(int nparts, const u64 *partials, ProofState *ps,
                                                  u64 *msg, u64 *chal, int last, const u64 *Flast,
                                                  u64 *vout) {
    u64 t[4];
    rows_total<4>(nparts, partials, t);
    if (threadIdx.x == 0) {
        const u64 E0 = t[0], E1 = t[1], O0 = t[2], O1 = t[3];
        msg[0] = E0;
        msg[1] = O1;
        u64 o4 = add(O1, O1);
        o4 = add(o4, o4);
        msg[2] = sub(add(sub(E0, add(E1, E1)), o4), add(O0, O0));
        const u64 r = draw(ps);
        *chal = r;
        if (last) {
            const u64 f0 = Flast[0], f1 = Flast[1];
            const u64 v = add(f0, mul(r, sub(f1, f0)));
            *vout = v;
            if (last == 1) ps->v1 = v;
        }
    }
}

hipError_t launch_wfinal(hipStream_t st, int nparts, const u64 *partials, ProofState *ps, u64 *msg,
                         u64 *chal, int last, const u64 *Flast, u64 *vout) {
    hipLaunchKernelGGL(k_wfinal, dim3(1), dim3(BLOCK), 0, st, nparts, partials, ps, msg, chal, last,
                       Flast, vout);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_fold(u64 nh, const u64 *src, u64 *dst, const u64 *rptr) {
    const u64 r = *rptr;
    for (u64 m = GTID; m < nh; m += GSTRIDE) {
        const u64x2 p = ld2(src, 2 * m);
        dst[m] = add(p.x, mul(r, sub(p.y, p.x)));
    }
}

hipError_t launch_fold(hipStream_t st, u64 nh, const u64 *src, u64 *dst, const u64 *rptr) {
    hipLaunchKernelGGL(k_fold, dim3(blocks_for(nh, 4)), dim3(BLOCK), 0, st, nh, src, dst, rptr);
    return hipGetLastError();
}

__global__ void k_single_gate_end(const u64 *Vn, ProofState *ps, u64 *msg_v) {
    if (threadIdx.x == 0) {
        const u64 v = Vn[0];
        msg_v[0] = v;
        msg_v[1] = v;
        ps->v1 = v;
    }
}

hipError_t launch_single_gate_end(hipStream_t st, const u64 *Vn, ProofState *ps, u64 *msg_v) {
    hipLaunchKernelGGL(k_single_gate_end, dim3(1), dim3(64), 0, st, Vn, ps, msg_v);
    return hipGetLastError();
}

// ------------------------------------------------------------ line step (a9)
//
// h(t) = ~V_{i+1}(l(t)) for t = 2..s', l(t) = b* + t (c* - b*), T = s' - 1
// points.  The index splits as x = (hh 2^M + mid) 2^L + lane with L <= 6
// and 2^M the number of waves: chi_x(l(t)) = Hh_t[hh] Hl_t[mid] lo_t[lane].
// Wave `mid` walks hh accumulating Hh_t[hh] V[x] for each t (one product
// per element and point), and multiplies by Hl_t[mid] lo_t[lane] once.
// Tables: lo [T][2^L], Hl [T][2^M], Hh [2^{s'-L-M}][T] (a step's T weights
// contiguous).

__global__ void __launch_bounds__(BLOCK) k_line_tables(const u64 *bstar, const u64 *cstar, u32 sp,
                                                       u32 L, u32 M, u64 *lo, u64 *hl, u64 *hh) {
    const u32 T = sp - 1, H = sp - L - M;
    const u64 nlo = 1ull << L, nhl = 1ull << M, nhh = 1ull << H;
    const u64 per = nlo + nhl + nhh;
    for (u64 e = GTID; e < (u64)T * per; e += GSTRIDE) {
        const u32 tp = (u32)(e / per);
        const u64 x = e % per;
        const u64 t = tp + 2;
        u32 base, n;
        u64 bits;
        if (x < nlo) {
            base = 0; n = L; bits = x;
        } else if (x < nlo + nhl) {
            base = L; n = M; bits = x - nlo;
        } else {
            base = L + M; n = H; bits = x - nlo - nhl;
        }
        u64 v = 1;
        for (u32 k = 0; k < n; k++) {
            const u64 b = bstar[base + k], c = cstar[base + k];
            const u64 l = add(b, mul(t, sub(c, b)));
            v = mul(v, fp::eqbit((u32)((bits >> k) & 1), l));
        }
        if (x < nlo)
            lo[(u64)tp * nlo + bits] = v;
        else if (x < nlo + nhl)
            hl[(u64)tp * nhl + bits] = v;
        else
            hh[bits * T + tp] = v;
    }
}

hipError_t launch_line_tables(hipStream_t st, const u64 *bstar, const u64 *cstar, u32 sp, u32 L,
                              u32 M, u64 *lo, u64 *hl, u64 *hh) {
    const u64 n = (u64)(sp - 1) * ((1ull << L) + (1ull << M) + (1ull << (sp - L - M)));
    hipLaunchKernelGGL(k_line_tables, dim3(blocks_for(n)), dim3(BLOCK), 0, st, bstar, cstar, sp, L,
                       M, lo, hl, hh);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_line(u32 sp, u32 L, u32 M, const u64 *V, const u64 *lo,
                                                const u64 *hl, const u64 *hh, u64 *partials) {
    const u32 T = sp - 1, H = sp - L - M;
    const u64 nlo = 1ull << L, nhl = 1ull << M, nhh = 1ull << H;
    const u32 lane = threadIdx.x & 63;
    const u64 mid = (u64)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    u64 acc[MAX_LINE];
#pragma unroll
    for (int t = 0; t < MAX_LINE; t++) acc[t] = 0;
    if (lane < nlo && mid < nhl) {
        for (u64 h = 0; h < nhh; h++) {
            const u64 v = V[(((h << M) + mid) << L) + lane];
            const u64 *w = hh + h * T;
#pragma unroll
            for (int t = 0; t < MAX_LINE; t++)
                if (t < (int)T) acc[t] = add(acc[t], mul(w[t], v));
        }
#pragma unroll
        for (int t = 0; t < MAX_LINE; t++)
            if (t < (int)T)
                acc[t] = mul(acc[t], mul(hl[(u64)t * nhl + mid], lo[(u64)t * nlo + lane]));
    }
    block_store<MAX_LINE>(acc, partials + (u64)blockIdx.x * MAX_LINE);
}

hipError_t launch_line(hipStream_t st, u32 sp, u32 L, u32 M, const u64 *V, const u64 *lo,
                       const u64 *hl, const u64 *hh, u64 *partials, int *nblocks) {
    const u64 nwaves = 1ull << M;
    int nb = (int)((nwaves + (BLOCK / 64) - 1) / (BLOCK / 64));
    *nblocks = nb;
    hipLaunchKernelGGL(k_line, dim3(nb), dim3(BLOCK), 0, st, sp, L, M, V, lo, hl, hh, partials);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_line_final(int nparts, const u64 *partials, u32 sp,
                                                      ProofState *ps, const u64 *bstar,
                                                      const u64 *cstar, u64 *msg, u64 *chal,
                                                      u64 *zbuf) {
    u64 t[MAX_LINE];
    rows_total<MAX_LINE>(nparts, partials, t);
    if (threadIdx.x == 0) {
        for (u32 k = 2; k <= sp; k++) msg[k - 2] = t[k - 2];
        const u64 tau = draw(ps);
        *chal = tau;
        for (u32 k = 0; k < sp; k++) {
            const u64 b = bstar[k], c = cstar[k];
            zbuf[k] = add(b, mul(tau, sub(c, b)));
        }
        ps->betaC = 1;  // the next layer's a-variables start unbound
    }
}

hipError_t launch_line_final(hipStream_t st, int nparts, const u64 *partials, u32 sp,
                             ProofState *ps, const u64 *bstar, const u64 *cstar, u64 *msg,
                             u64 *chal, u64 *zbuf) {
    hipLaunchKernelGGL(k_line_final, dim3(1), dim3(BLOCK), 0, st, nparts, partials, sp, ps, bstar,
                       cstar, msg, chal, zbuf);
    return hipGetLastError();
}

// ---------------------------------------------------------- verifier (a10)

template <int KIND>
__global__ void __launch_bounds__(BLOCK) k_wiring(WiringArgs a) {
    const u64 am = (1ull << a.La) - 1, bm = (1ull << a.Lb) - 1, cm = (1ull << a.Lc) - 1;
    u64 acc[2] = {0, 0};
    for (u64 g = GTID; g < a.S; g += GSTRIDE) {
        const u32 i1 = a.in1[g], i2 = a.in2[g];
        const u64 ea = mul(a.alo[g & am], a.ahi[g >> a.La]);
        const u64 eb = mul(a.blo[i1 & bm], a.bhi[i1 >> a.Lb]);
        const u64 ec = mul(a.clo[i2 & cm], a.chi[i2 >> a.Lc]);
        const u64 e = mul(ea, mul(eb, ec));
        const bool ismul = KIND == KIND_MUL || (KIND == KIND_MIXED && a.type[g]);
        if (ismul)
            acc[1] = add(acc[1], e);
        else
            acc[0] = add(acc[0], e);
    }
    block_store<2>(acc, a.partials + 2 * (u64)blockIdx.x);
}

hipError_t launch_wiring(hipStream_t st, const WiringArgs &a, int *nblocks) {
    int nb = blocks_for(a.S, 4);
    *nblocks = nb;
    dim3 g(nb), b(BLOCK);
    if (a.kind == KIND_ADD) hipLaunchKernelGGL(k_wiring<KIND_ADD>, g, b, 0, st, a);
    else if (a.kind == KIND_MUL) hipLaunchKernelGGL(k_wiring<KIND_MUL>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_wiring<KIND_MIXED>, g, b, 0, st, a);
    return hipGetLastError();
}

template <bool WIDE>
__global__ void __launch_bounds__(BLOCK) k_mle(u64 n, const u64 *T64, const u32 *T32, const u64 *lo,
                                               const u64 *hi, u32 L, u64 *partials) {
    const u64 mask = (1ull << L) - 1;
    u64 acc[1] = {0};
    for (u64 x = GTID; x < n; x += GSTRIDE) {
        const u64 v = WIDE ? T64[x] : (u64)T32[x];
        acc[0] = add(acc[0], mul(mul(lo[x & mask], hi[x >> L]), v));
    }
    block_store<1>(acc, partials + (u64)blockIdx.x);
}

hipError_t launch_mle(hipStream_t st, u64 n, const u64 *T64, const u32 *T32, const u64 *lo,
                      const u64 *hi, u32 L, u64 *partials, int *nblocks) {
    int nb = blocks_for(n, 8);
    *nblocks = nb;
    if (T64)
        hipLaunchKernelGGL(k_mle<true>, dim3(nb), dim3(BLOCK), 0, st, n, T64, T32, lo, hi, L, partials);
    else
        hipLaunchKernelGGL(k_mle<false>, dim3(nb), dim3(BLOCK), 0, st, n, T64, T32, lo, hi, L,
                           partials);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_reduce_rows(int nparts, int K, const u64 *partials, u64 *out) {
    u64 v[4] = {0, 0, 0, 0};
    for (int r = threadIdx.x; r < nparts; r += BLOCK)
        for (int k = 0; k < K; k++) v[k] = add(v[k], partials[(u64)r * K + k]);
    __shared__ u64 res[4];
    block_store<4>(v, res);
    __syncthreads();
    if (threadIdx.x < K) out[threadIdx.x] = res[threadIdx.x];
}

hipError_t launch_reduce_rows(hipStream_t st, int nparts, int K, const u64 *partials, u64 *out) {
    hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(BLOCK), 0, st, nparts, K, partials, out);
    return hipGetLastError();
}

// ------------------------------------------------------- F2 sum-check (a11)

template <int J>  // 0: first round, 1: second round (u32 source), 2: later rounds
__global__ void __launch_bounds__(BLOCK) k_f2sc_round(u64 nm, const u32 *a32, const u64 *Asrc,
                                                      u64 *Aout, const u64 *rptr, u64 *partials) {
    u64 r = 0;
    if (J > 0) r = *rptr;
    u64 acc[3] = {0, 0, 0};
    for (u64 m = GTID; m < nm; m += GSTRIDE) {
        u64 v0, v1;
        if (J == 0) {
            const uint2 p = *reinterpret_cast<const uint2 *>(a32 + 2 * m);
            v0 = p.x;
            v1 = p.y;
        } else if (J == 1) {
            const uint4 p = *reinterpret_cast<const uint4 *>(a32 + 4 * m);
            v0 = add(p.x, mul(r, sub(p.y, p.x)));
            v1 = add(p.z, mul(r, sub(p.w, p.z)));
            st2(Aout, 2 * m, v0, v1);
        } else {
            const u64x2 p = ld2(Asrc, 4 * m), q = ld2(Asrc, 4 * m + 2);
            v0 = add(p.x, mul(r, sub(p.y, p.x)));
            v1 = add(q.x, mul(r, sub(q.y, q.x)));
            st2(Aout, 2 * m, v0, v1);
        }
        const u64 d = sub(add(v1, v1), v0);
        acc[0] = add(acc[0], mul(v0, v0));
        acc[1] = add(acc[1], mul(v1, v1));
        acc[2] = add(acc[2], mul(d, d));
    }
    block_store<3>(acc, partials + 3 * (u64)blockIdx.x);
}

hipError_t launch_f2sc_round(hipStream_t st, int j, u64 nm, const u32 *a32, const u64 *Asrc,
                             u64 *Aout, const u64 *rptr, u64 *partials, int *nblocks) {
    int nb = blocks_for(nm, 4);
    *nblocks = nb;
    dim3 g(nb), b(BLOCK);
    if (j == 0) hipLaunchKernelGGL(k_f2sc_round<0>, g, b, 0, st, nm, a32, Asrc, Aout, rptr, partials);
    else if (j == 1) hipLaunchKernelGGL(k_f2sc_round<1>, g, b, 0, st, nm, a32, Asrc, Aout, rptr, partials);
    else hipLaunchKernelGGL(k_f2sc_round<2>, g, b, 0, st, nm, a32, Asrc, Aout, rptr, partials);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_f2sc_final(int nparts, const u64 *partials, ProofState *ps,
                                                      u64 *msg, u64 *chal, u64 *f2) {
    u64 t[3];
    rows_total<3>(nparts, partials, t);
    if (threadIdx.x == 0) {
        msg[0] = t[0];
        msg[1] = t[1];
        msg[2] = t[2];
        if (f2) *f2 = add(t[0], t[1]);
        *chal = draw(ps);
    }
}

hipError_t launch_f2sc_final(hipStream_t st, int nparts, const u64 *partials, ProofState *ps,
                             u64 *msg, u64 *chal, u64 *f2) {
    hipLaunchKernelGGL(k_f2sc_final, dim3(1), dim3(BLOCK), 0, st, nparts, partials, ps, msg, chal, f2);
    return hipGetLastError();
}

__global__ void k_f2sc_init(ProofState *ps, u64 seed) {
    if (threadIdx.x == 0) {
        ps->rng = fp::sm_state(seed, fp::PURPOSE_F2SC);
        ps->betaC = 1;
        ps->v1 = 0;
    }
}

hipError_t launch_f2sc_init(hipStream_t st, ProofState *ps, u64 seed) {
    hipLaunchKernelGGL(k_f2sc_init, dim3(1), dim3(64), 0, st, ps, seed);
    return hipGetLastError();
}

__global__ void k_f2sc_single(const u32 *a32, u64 *msg) {
    if (threadIdx.x == 0) {
        const u64 v = a32[0];
        msg[0] = mul(v, v);
    }
}

hipError_t launch_f2sc_single(hipStream_t st, const u32 *a32, u64 *msg) {
    hipLaunchKernelGGL(k_f2sc_single, dim3(1), dim3(64), 0, st, a32, msg);
    return hipGetLastError();
}

// ------------------------------------------------------------ field check

__global__ void __launch_bounds__(BLOCK) k_field_op(int op, const u64 *a, const u64 *b, u64 *out,
                                                    u64 n) {
    for (u64 i = GTID; i < n; i += GSTRIDE) {
        const u64 x = a[i], y = b[i];
        out[i] = op == 0 ? add(x, y) : (op == 1 ? sub(x, y) : mul(x, y));
    }
}

hipError_t launch_field_op(hipStream_t st, int op, const u64 *a, const u64 *b, u64 *out, u64 n) {
    hipLaunchKernelGGL(k_field_op, dim3(blocks_for(n, 4)), dim3(BLOCK), 0, st, op, a, b, out, n);
    return hipGetLastError();
}

}  // namespace gkr
