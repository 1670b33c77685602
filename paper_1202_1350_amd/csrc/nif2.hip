// nif2.hip -- the non-interactive F2 protocol (Sec. 3.2, 4.2) on
// gfx950: the prover's prime factor transforms of the grid rows and the
// column square-sums of its proof, and the verifier's row evaluations.
//
// The universe is a v x h grid, cell (row y, column j) = a_{j v + y}, so
// element j of every row is one contiguous run of v words: a thread per
// (row, line of a pass) reads and writes coalesced, the layout the paper
// reaches by transposing the grid (Sec. 6.2.1).  Row y is the polynomial
// f_y of degree < h through the order-h subgroup H = <w>; the proof is
// g = sum_y f_y^2 on the order-2h subgroup <xi> (xi^2 = w): the even points
// are the data squared, the odd points are f_y on the coset xi H, obtained
// from an inverse transform (values -> coefficients c), a twist
// c_k xi^k / h and a forward transform.
#include "fp61.hpp"
#include "nif2.hpp"

namespace gkr {

using fp::add;
using fp::mul;
using fp::P;
using fp::sub;
using fp::u128;

constexpr int NT = 256;  // threads per workgroup of these kernels

struct PassArgs {
    PfaPlan pl;
    u64 n, v;
    u32 dim;       // digit transformed by this pass
    u64 wp[25];    // powers 0 .. F-1 of the pass's root
};

__device__ __forceinline__ u32 good_index(const PfaPlan &pl, u64 pos) {
    u64 g = 0;
    for (u32 i = 0; i < pl.nf; i++) g += (pos / pl.stride[i]) % pl.F[i] * pl.gstep[i];
    return (u32)(g % pl.h);
}
__device__ __forceinline__ u32 crt_index(const PfaPlan &pl, u64 pos) {
    u64 c = 0;
    for (u32 i = 0; i < pl.nf; i++) c += (pos / pl.stride[i]) % pl.F[i] * pl.cstep[i];
    return (u32)(c % pl.h);
}

// One pass: the F-point DFT along digit `dim` of every line of every row.
// MODE 1 gathers the row from a in Good order (the first inverse pass);
// MODE 2 twists by tw[CRT(position)] as it loads (the first forward pass).
template <int F, int MODE>
__global__ void __launch_bounds__(NT) k_pfa_pass(const PassArgs pa, const u64 *__restrict__ a,
                                                 const u64 *__restrict__ tw, u64 *W) {
    const PfaPlan &pl = pa.pl;
    const u64 v = pa.v, s = pl.stride[pa.dim];
    const u64 total = (u64)(pl.h / F) * v;
    for (u64 gid = (u64)blockIdx.x * NT + threadIdx.x; gid < total; gid += (u64)gridDim.x * NT) {
        const u64 y = gid % v, l = gid / v;
        const u64 base = (l % s) + (l / s) * s * F;
        u64 x[F];
        if (MODE == 1) {
            const u32 g0 = good_index(pl, base), gs = pl.gstep[pa.dim];
#pragma unroll
            for (int m = 0; m < F; m++) {
                const u64 j = (g0 + (u64)m * gs) % pl.h, i = j * v + y;
                x[m] = i < pa.n ? a[i] : 0;
            }
        } else if (MODE == 2) {
            const u32 c0 = crt_index(pl, base), cs = pl.cstep[pa.dim];
#pragma unroll
            for (int m = 0; m < F; m++)
                x[m] = mul(W[(base + m * s) * v + y], tw[(c0 + (u64)m * cs) % pl.h]);
        } else {
#pragma unroll
            for (int m = 0; m < F; m++) x[m] = W[(base + m * s) * v + y];
        }
        if constexpr (F == 25) {
            // 25 = 5 x 5: n = 5 n1 + n2, k = k1 + 5 k2, w^{nk} = u^{n1 k1} w^{n2 k1} u^{n2 k2}
            // with u = w^5: five 5-point DFTs over n1 (in place), twiddles w^{n2 k1},
            // five 5-point DFTs over n2 written out
#pragma unroll
            for (int n2 = 0; n2 < 5; n2++) {
                u64 t[5];
#pragma unroll
                for (int k1 = 0; k1 < 5; k1++) {
                    u128 acc = 0;
#pragma unroll
                    for (int n1 = 0; n1 < 5; n1++) acc += fp::wide(x[5 * n1 + n2], pa.wp[(5 * n1 * k1) % 25]);
                    t[k1] = fp::red128(acc);
                }
#pragma unroll
                for (int k1 = 0; k1 < 5; k1++) x[5 * k1 + n2] = (n2 * k1) ? mul(t[k1], pa.wp[n2 * k1]) : t[k1];
            }
#pragma unroll
            for (int k1 = 0; k1 < 5; k1++) {
#pragma unroll
                for (int k2 = 0; k2 < 5; k2++) {
                    u128 acc = 0;
#pragma unroll
                    for (int n2 = 0; n2 < 5; n2++) acc += fp::wide(x[5 * k1 + n2], pa.wp[(5 * n2 * k2) % 25]);
                    W[(base + (k1 + 5 * k2) * s) * v + y] = fp::red128(acc);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < F; k++) {
                u128 acc = 0;
#pragma unroll
                for (int m = 0; m < F; m++) acc += fp::wide(x[m], pa.wp[(m * k) % F]);  // F < 32 terms < 2^127
                W[(base + k * s) * v + y] = fp::red128(acc);
            }
        }
    }
}

static u32 grid_of(u64 items) {
    const u64 b = (items + NT - 1) / NT;
    return (u32)std::max<u64>(1, std::min<u64>(b, 4096));
}

template <int MODE>
static hipError_t pass(hipStream_t st, const PassArgs &pa, const u64 *a, const u64 *tw, u64 *W) {
    const u32 F = pa.pl.F[pa.dim];
    const dim3 g(grid_of((u64)(pa.pl.h / F) * pa.v)), b(NT);
    switch (F) {
#define PF(N) case N: hipLaunchKernelGGL((k_pfa_pass<N, MODE>), g, b, 0, st, pa, a, tw, W); break;
        PF(3) PF(5) PF(7) PF(9) PF(11) PF(13) PF(25)
#undef PF
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_nif2_transform(hipStream_t st, const PfaPlan &pl, const u64 *a, u64 n, u64 v,
                                 const u64 *tw, u64 *W) {
    PassArgs pa;
    pa.pl = pl;
    pa.n = n;
    pa.v = v;
    // inverse transform: values on H (Good order) -> coefficients (CRT order)
    for (u32 d = 0; d < pl.nf; d++) {
        pa.dim = d;
        u64 w = 1;
        for (u32 m = 0; m < pl.F[d]; m++, w = mul(w, pl.winv[d])) pa.wp[m] = w;
        const hipError_t e = d == 0 ? pass<1>(st, pa, a, tw, W) : pass<0>(st, pa, a, tw, W);
        if (e != hipSuccess) return e;
    }
    // twist by xi^k / h, forward transform: CRT order -> f_y(xi w^j) in Good order
    for (u32 d = 0; d < pl.nf; d++) {
        pa.dim = d;
        u64 w = 1;
        for (u32 m = 0; m < pl.F[d]; m++, w = mul(w, pl.wfwd[d])) pa.wp[m] = w;
        const hipError_t e = d == 0 ? pass<2>(st, pa, a, tw, W) : pass<0>(st, pa, a, tw, W);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ reductions

// Workgroup sum of one value per thread, returned to thread 0.
__device__ __forceinline__ u64 group_sum(u64 v) {
    __shared__ u64 sm[NT / 64];
    for (int o = 32; o > 0; o >>= 1) {
        const int lo = __shfl_down((int)(u32)v, o), hi = __shfl_down((int)(u32)(v >> 32), o);
        v = add(v, ((u64)(u32)hi << 32) | (u32)lo);
    }
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    u64 t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; w++) t = add(t, sm[w]);
    return t;
}

// Sum of squares of `cnt` words at src[0 .. cnt) (only i < lim count), in
// u128 with a reduction every 16 terms.
__device__ __forceinline__ u64 sq_sum(const u64 *src, u64 cnt, u64 off, u64 lim) {
    u64 s = 0;
    u128 acc = 0;
    u32 t = 0;
    for (u64 y = threadIdx.x; y < cnt; y += NT) {
        const u64 x = off + y < lim ? src[y] : 0;
        acc += fp::wide(x, x);
        if (++t == 16) {
            s = add(s, fp::red128(acc));
            acc = 0;
            t = 0;
        }
    }
    return add(s, fp::red128(acc));
}

// Workgroup (k, c): the part of g(xi^k) = sum_y (value k of row y)^2 over
// rows [c ch, (c + 1) ch), into part[k S + c].
__global__ void __launch_bounds__(NT) k_nif2_colsum(const PfaPlan pl, const u64 *__restrict__ a, u64 n, u64 v,
                                                    const u64 *__restrict__ W, u64 ch, u32 S, u64 *part) {
    const u32 k = blockIdx.x / S, c = blockIdx.x % S;
    const u64 y0 = c * ch, cnt = y0 < v ? std::min<u64>(ch, v - y0) : 0;
    const u64 j = k >> 1;
    u64 s;
    if ((k & 1) == 0) {
        s = sq_sum(a + j * v + y0, cnt, j * v + y0, n);
    } else {
        u64 pos = 0;  // f_y(xi w^j) sits at the position whose Good index is j
        for (u32 i = 0; i < pl.nf; i++) pos += (j * pl.ginv[i] % pl.F[i]) * pl.stride[i];
        s = sq_sum(W + pos * v + y0, cnt, 0, cnt);
    }
    s = group_sum(s);
    if (threadIdx.x == 0) part[(u64)k * S + c] = s;
}

// msgs[k] = sum_c part[k S + c]
__global__ void k_nif2_colfin(const u64 *__restrict__ part, u32 S, u32 K, u64 *msgs) {
    const u32 k = blockIdx.x * NT + threadIdx.x;
    if (k >= K) return;
    u64 s = 0;
    for (u32 c = 0; c < S; c++) s = add(s, part[(u64)k * S + c]);
    msgs[k] = s;
}

u32 nif2_colsum_split(u32 h, u64 v) {
    // about 2048 workgroups in all, each over at least 4096 rows
    const u64 want = std::max<u64>(1, 2048 / (2ull * h));
    return (u32)std::max<u64>(1, std::min<u64>(want, v / 4096));
}

hipError_t launch_nif2_colsum(hipStream_t st, const PfaPlan &pl, const u64 *a, u64 n, u64 v, const u64 *W,
                              u64 *part, u64 *msgs) {
    const u32 S = nif2_colsum_split(pl.h, v);
    const u64 ch = (v + S - 1) / S;
    hipLaunchKernelGGL(k_nif2_colsum, dim3(2 * pl.h * S), dim3(NT), 0, st, pl, a, n, v, W, ch, S, part);
    hipLaunchKernelGGL(k_nif2_colfin, dim3((2 * pl.h + NT - 1) / NT), dim3(NT), 0, st, part, S, 2 * pl.h, msgs);
    return hipGetLastError();
}

__global__ void k_nif2_twist(u32 h, u64 xi, u64 hinv, u64 *tw) {
    const u32 k = blockIdx.x * NT + threadIdx.x;
    if (k < h) tw[k] = mul(fp::pow(xi, k), hinv);
}

hipError_t launch_nif2_twist(hipStream_t st, u32 h, u64 xi, u64 *tw) {
    hipLaunchKernelGGL(k_nif2_twist, dim3((h + NT - 1) / NT), dim3(NT), 0, st, h, xi, fp::inv(h), tw);
    return hipGetLastError();
}

// ------------------------------------------------------------- verifier

// L[j] = w^j (r^N - 1) / (N (r - w^j)), or [w^j == r] when r^N = 1.
__global__ void k_nif2_basis(u64 w, u64 N, u64 r, u64 rN1, u64 *L) {
    const u64 j = (u64)blockIdx.x * NT + threadIdx.x;
    if (j >= N) return;
    const u64 wj = fp::pow(w, j);
    if (rN1 == 0) {
        L[j] = wj == r ? 1 : 0;
        return;
    }
    L[j] = mul(mul(wj, rN1), fp::inv(mul(N % P, sub(r, wj))));
}

hipError_t launch_nif2_basis(hipStream_t st, u64 w, u64 N, u64 r, u64 *L) {
    const u64 rN1 = sub(fp::pow(r, N), 1);
    hipLaunchKernelGGL(k_nif2_basis, dim3((u32)((N + NT - 1) / NT)), dim3(NT), 0, st, w, N, r, rN1, L);
    return hipGetLastError();
}

constexpr u32 RCH = 32;  // columns per partial row evaluation (32 products < 2^127)

// part[c v + y] = sum_{j in chunk c} a(j, y) L[j]
__global__ void __launch_bounds__(NT) k_nif2_rowpart(const u64 *__restrict__ a, u64 n, u64 v, u32 h,
                                                     const u64 *__restrict__ L, u64 *part) {
    const u64 nch = (h + RCH - 1) / RCH, total = nch * v;
    for (u64 gid = (u64)blockIdx.x * NT + threadIdx.x; gid < total; gid += (u64)gridDim.x * NT) {
        const u64 y = gid % v, c = gid / v;
        u128 acc = 0;
        for (u64 j = c * RCH; j < std::min<u64>(h, (c + 1) * RCH); j++) {
            const u64 i = j * v + y;
            acc += fp::wide(i < n ? a[i] : 0, L[j]);
        }
        part[c * v + y] = fp::red128(acc);
    }
}

// blk[b] = sum over this workgroup's rows y of (sum_c part[c v + y])^2
__global__ void __launch_bounds__(NT) k_nif2_rowsq(const u64 *__restrict__ part, u64 v, u32 nch, u64 *blk) {
    u64 s = 0;
    for (u64 y = (u64)blockIdx.x * NT + threadIdx.x; y < v; y += (u64)gridDim.x * NT) {
        u64 t = 0;
        for (u32 c = 0; c < nch; c++) t = add(t, part[(u64)c * v + y]);
        s = add(s, mul(t, t));
    }
    s = group_sum(s);
    if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

__global__ void __launch_bounds__(NT) k_nif2_sum(const u64 *__restrict__ x, u64 cnt, u64 *out) {
    u64 s = 0;
    for (u64 i = threadIdx.x; i < cnt; i += NT) s = add(s, x[i]);
    s = group_sum(s);
    if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_nif2_rows(hipStream_t st, const u64 *a, u64 n, u64 v, u32 h, const u64 *L, u64 *part,
                            u64 *blk, u64 *out) {
    const u32 nch = (h + RCH - 1) / RCH;
    hipLaunchKernelGGL(k_nif2_rowpart, dim3(grid_of((u64)nch * v)), dim3(NT), 0, st, a, n, v, h, L, part);
    const u32 nb = (u32)std::min<u64>(1024, (v + NT - 1) / NT);
    hipLaunchKernelGGL(k_nif2_rowsq, dim3(nb), dim3(NT), 0, st, part, v, nch, blk);
    hipLaunchKernelGGL(k_nif2_sum, dim3(1), dim3(NT), 0, st, blk, (u64)nb, out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(NT) k_nif2_dot(const u64 *__restrict__ x, const u64 *__restrict__ y, u64 N,
                                                 u64 *blk) {
    u64 s = 0;
    for (u64 k = (u64)blockIdx.x * NT + threadIdx.x; k < N; k += (u64)gridDim.x * NT) s = add(s, mul(x[k], y[k]));
    s = group_sum(s);
    if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

hipError_t launch_nif2_dot(hipStream_t st, const u64 *msgs, const u64 *L2, u64 N, u64 *blk, u64 *out) {
    const u32 nb = (u32)std::min<u64>(1024, (N + NT - 1) / NT);
    hipLaunchKernelGGL(k_nif2_dot, dim3(nb), dim3(NT), 0, st, msgs, L2, N, blk);
    hipLaunchKernelGGL(k_nif2_sum, dim3(1), dim3(NT), 0, st, blk, (u64)nb, out);
    return hipGetLastError();
}

__global__ void k_nif2_range(const u64 *__restrict__ a, u64 n, u32 *flag) {
    for (u64 i = (u64)blockIdx.x * NT + threadIdx.x; i < n; i += (u64)gridDim.x * NT)
        if (a[i] >= P) flag[0] = 1;
}

hipError_t launch_nif2_range(hipStream_t st, const u64 *a, u64 n, u32 *flag) {
    hipLaunchKernelGGL(k_nif2_range, dim3(grid_of(n)), dim3(NT), 0, st, a, n, flag);
    return hipGetLastError();
}

}  // namespace gkr
