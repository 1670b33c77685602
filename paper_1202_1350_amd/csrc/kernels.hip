// kernels.hip -- HIP kernels (gfx950) of the GKR prover's per-layer
// sum-check over F_p, p = 2^61 - 1, of its verifier, and of the F2
// sum-check.
//
// Sec. 4.1.1: each gate contributes independently to the prover's message;
// a workgroup sums its gates' contributions (wave64 shuffles, then LDS),
// writes one row of partial sums, and a one-workgroup *_final kernel folds
// the rows, writes the message and only then draws the next challenge on
// the device.  All arithmetic is exact modular integer arithmetic (no
// floating point, Sec. 6.1), so any summation order gives identical bits.
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

// Challenge d of the F2 sum-check, drawn from the state before it; the
// state after it goes to *next when not NULL.
__device__ __forceinline__ u64 draw(const ProofState *ps, int d, u64 *next) {
    u64 s = ps->rng[d & 1];
    const u64 r = fp::sm_field(s);
    if (next) *next = s;
    return r;
}

// Message of F2 sum-check round d from its partial rows, challenge r_d, and
// the state after it (one workgroup).
__device__ __forceinline__ void f2sc_finish(int d, int nparts, const u64 *part, ProofState *ps, u64 *msg,
                                            u64 *chal, u64 *f2) {
    u64 t[3];
    rows_total<3>(nparts, part, t);
    if (threadIdx.x == 0) {
        msg[0] = t[0];
        msg[1] = t[1];
        msg[2] = t[2];
        if (f2) *f2 = add(t[0], t[1]);
        *chal = draw(ps, d, &ps->rng[(d + 1) & 1]);
    }
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

// --------------------------------------------------------- proof bookkeeping

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
                                               const u64 *hi, u32 L, u64 *partials, int accumulate) {
    const u64 mask = (1ull << L) - 1;
    u64 acc[1] = {0};
    if ((GSTRIDE & mask) == 0) {
        // every x of this thread has the same low bits: chi_x = lo[x & mask]
        // hi[x >> L], so the thread sums hi[x >> L] v_x exactly in 128 bits
        // (reduced every 32 terms: 32 products below 2^122 fit) and
        // multiplies by its lo once
        u64 s = 0;
        fp::u128 w = 0;
        u32 k = 0;
        for (u64 x = GTID; x < n; x += GSTRIDE) {
            w += WIDE ? fp::wide(hi[x >> L], T64[x]) : fp::wide(hi[x >> L], (u64)T32[x]);
            if (++k == 32) {
                s = add(s, fp::red128(w));
                w = 0;
                k = 0;
            }
        }
        s = add(s, fp::red128(w));
        acc[0] = GTID < n ? mul(s, lo[GTID & mask]) : 0;
    } else {
        for (u64 x = GTID; x < n; x += GSTRIDE) {
            const u64 v = WIDE ? T64[x] : (u64)T32[x];
            acc[0] = add(acc[0], mul(mul(lo[x & mask], hi[x >> L]), v));
        }
    }
    __shared__ u64 tot[1];
    block_store<1>(acc, tot);
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = accumulate ? add(partials[blockIdx.x], tot[0]) : tot[0];
}

hipError_t launch_mle(hipStream_t st, u64 n, const u64 *T64, const u32 *T32, const u64 *lo,
                      const u64 *hi, u32 L, u64 *partials, int *nblocks, int accumulate, int nb_fixed) {
    const int nb = nb_fixed > 0 ? nb_fixed : blocks_for(n, 8);
    *nblocks = nb;
    if (T64)
        hipLaunchKernelGGL(k_mle<true>, dim3(nb), dim3(BLOCK), 0, st, n, T64, T32, lo, hi, L, partials,
                           accumulate);
    else
        hipLaunchKernelGGL(k_mle<false>, dim3(nb), dim3(BLOCK), 0, st, n, T64, T32, lo, hi, L,
                           partials, accumulate);
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
__global__ void __launch_bounds__(BLOCK) k_f2sc_round(int j, u64 nm, const u32 *a32, const u64 *Asrc,
                                                      u64 *Aout, ProofState *ps, u64 *part, int prev_parts,
                                                      u64 *prev_msg, u64 *prev_chal, u64 *f2) {
    const u32 nb = gridDim.x - (J > 0 ? 1 : 0);  // body workgroups
    if (J > 0 && blockIdx.x == nb) {  // finishes round j - 1 beside the body
        f2sc_finish(j - 1, prev_parts, part + 3ull * MAX_BLOCKS * ((j - 1) & 1), ps, prev_msg, prev_chal, f2);
        return;
    }
    u64 r = 0;
    if (J > 0) r = draw(ps, j - 1, nullptr);  // r_{j-1}: round j-1's sums are complete
    const u64 stride = (u64)nb * BLOCK;
    u64 acc[3] = {0, 0, 0};
    if (J == 0) {
        // u32 pairs (a, b): a^2, b^2 and ab are exact in 64 bits; their sums
        // stay exact in 128 bits (a thread adds far fewer than 2^64 terms), and
        // (2b - a)^2 = a^2 + 4 b^2 - 4 ab, so the thread reduces mod p once
        fp::u128 saa = 0, sbb = 0, sab = 0;
        for (u64 m = GTID; m < nm; m += stride) {
            const uint2 p = *reinterpret_cast<const uint2 *>(a32 + 2 * m);
            const u64 a = p.x, b = p.y;
            saa += a * a;
            sbb += b * b;
            sab += a * b;
        }
        const u64 ra = fp::red128(saa), rb = fp::red128(sbb), rab = fp::red128(sab);
        const u64 rb4 = add(add(rb, rb), add(rb, rb)), rab4 = add(add(rab, rab), add(rab, rab));
        acc[0] = ra;
        acc[1] = rb;
        acc[2] = sub(add(ra, rb4), rab4);
    }
    for (u64 m = GTID; J > 0 && m < nm; m += stride) {
        u64 v0, v1;
        if (J == 1) {
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
    block_store<3>(acc, part + 3ull * MAX_BLOCKS * (j & 1) + 3 * (u64)blockIdx.x);
}

hipError_t launch_f2sc_round(hipStream_t st, int j, u64 nm, const u32 *a32, const u64 *Asrc,
                             u64 *Aout, ProofState *ps, u64 *part, int prev_parts, u64 *prev_msg,
                             u64 *prev_chal, u64 *f2, int *nblocks) {
    const int nb = blocks_for(nm, 4);
    *nblocks = nb;
    const dim3 b(BLOCK);
    if (j == 0)
        hipLaunchKernelGGL(k_f2sc_round<0>, dim3(nb), b, 0, st, j, nm, a32, Asrc, Aout, ps, part, prev_parts,
                           prev_msg, prev_chal, f2);
    else if (j == 1)
        hipLaunchKernelGGL(k_f2sc_round<1>, dim3(nb + 1), b, 0, st, j, nm, a32, Asrc, Aout, ps, part,
                           prev_parts, prev_msg, prev_chal, f2);
    else
        hipLaunchKernelGGL(k_f2sc_round<2>, dim3(nb + 1), b, 0, st, j, nm, a32, Asrc, Aout, ps, part,
                           prev_parts, prev_msg, prev_chal, f2);
    return hipGetLastError();
}

__global__ void __launch_bounds__(BLOCK) k_f2sc_final(int j, int nparts, const u64 *part, ProofState *ps,
                                                      u64 *msg, u64 *chal, u64 *f2) {
    f2sc_finish(j, nparts, part + 3ull * MAX_BLOCKS * (j & 1), ps, msg, chal, f2);
}

__global__ void __launch_bounds__(BLOCK) k_f2sc_tail(int j0, int l, const u64 *Asrc, int prev_parts,
                                                     const u64 *part, ProofState *ps, u64 *msgs, u64 *chals) {
    __shared__ __align__(16) u64 T[2][F2SC_TAIL];
    __shared__ u64 tot[3];
    const int d = j0 - 1;
    f2sc_finish(d, prev_parts, part + 3ull * MAX_BLOCKS * (d & 1), ps, msgs + 1 + 3 * d, chals + d, nullptr);
    u64 st = ps->rng[d & 1];
    const u64 r0 = fp::sm_field(st);  // r_{j0-1}: round j0-1's sums are complete
    u32 nt = 1u << (l - j0);          // entries of level j0
    for (u32 e = threadIdx.x; e < nt; e += BLOCK) {
        const u64x2 p = ld2(Asrc, 2 * e);
        T[0][e] = add(p.x, mul(r0, sub(p.y, p.x)));
    }
    __syncthreads();
    for (int j = j0, b = 0; j < l; j++, b ^= 1, nt >>= 1) {
        const u32 half = nt >> 1;
        u64 acc[3] = {0, 0, 0};
        for (u32 m = threadIdx.x; m < half; m += BLOCK) {
            const u64 v0 = T[b][2 * m], v1 = T[b][2 * m + 1], dd = sub(add(v1, v1), v0);
            acc[0] = add(acc[0], mul(v0, v0));
            acc[1] = add(acc[1], mul(v1, v1));
            acc[2] = add(acc[2], mul(dd, dd));
        }
        block_store<3>(acc, tot);
        __syncthreads();  // round j's message is complete
        if (threadIdx.x < 3) msgs[1 + 3 * j + threadIdx.x] = tot[threadIdx.x];
        const u64 r = fp::sm_field(st);
        if (threadIdx.x == 0) chals[j] = r;
        for (u32 m = threadIdx.x; m < half; m += BLOCK) {
            const u64 v0 = T[b][2 * m], v1 = T[b][2 * m + 1];
            T[b ^ 1][m] = add(v0, mul(r, sub(v1, v0)));
        }
        __syncthreads();  // the next level is complete (and tot is read)
    }
}

hipError_t launch_f2sc_tail(hipStream_t st, int j0, int l, const u64 *Asrc, int prev_parts, const u64 *part,
                            ProofState *ps, u64 *msgs, u64 *chals) {
    hipLaunchKernelGGL(k_f2sc_tail, dim3(1), dim3(BLOCK), 0, st, j0, l, Asrc, prev_parts, part, ps, msgs, chals);
    return hipGetLastError();
}

hipError_t launch_f2sc_final(hipStream_t st, int j, int nparts, const u64 *part, ProofState *ps,
                             u64 *msg, u64 *chal, u64 *f2) {
    hipLaunchKernelGGL(k_f2sc_final, dim3(1), dim3(BLOCK), 0, st, j, nparts, part, ps, msg, chal, f2);
    return hipGetLastError();
}

__global__ void k_f2sc_init(ProofState *ps, u64 seed) {
    if (threadIdx.x == 0) {
        ps->rng[0] = fp::sm_state(seed, fp::PURPOSE_F2SC);
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
        if (op == 4) {
            // 256 dependent products per element: independent chains across
            // elements, for measuring the product rate
            u64 x = a[i];
            const u64 y = b[i];
#pragma unroll 16
            for (int k = 0; k < 256; k++) x = mul(x, y);
            out[i] = x;
            continue;
        }
        if (op == 3) {
            fp::u128 s = 0;
            for (u64 j = 0; j < 64; j++) {
                const u64 k = (i + j) % n;
                s += fp::wide(a[k], b[k]);
            }
            out[i] = fp::red128(s);
            continue;
        }
        const u64 x = a[i], y = b[i];
        out[i] = op == 0 ? add(x, y) : (op == 1 ? sub(x, y) : mul(x, y));
    }
}

hipError_t launch_field_op(hipStream_t st, int op, const u64 *a, const u64 *b, u64 *out, u64 n) {
    hipLaunchKernelGGL(k_field_op, dim3(blocks_for(n, 4)), dim3(BLOCK), 0, st, op, a, b, out, n);
    return hipGetLastError();
}

}  // namespace gkr
