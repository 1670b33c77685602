/*
 * gkr_oracle.c -- plain CPU oracle for the GKR prover/verifier over F_p,
 * p = 2^61 - 1, and for the interactive sum-check on F2 = sum_x a(x)^2.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU path is checked against.  Only the test suite, the
 * smoke entry point and the CPU-baseline leg of the benchmark may build,
 * load or call it.  It shares no code, header or table with the GPU
 * library and includes nothing from it.
 *
 * What it follows (Thaler, Roberts, Mitzenmacher, Pfister, "Verifiable
 * Computation with Massively Parallel Interactive Proofs"):
 *   - Sec. 6.1: all arithmetic is exact in F_p with p = 2^61 - 1.  Here every
 *     product is reduced with a plain 128-bit remainder, not with the
 *     Mersenne shift trick, so the reduction is independent of the GPU's.
 *   - Sec. 3.1: the layered fan-in-2 circuit of ADD/MUL gates; one iteration
 *     per layer turns a claim about one layer into a claim about the next,
 *     touching only those two layers.  Challenges are random field elements,
 *     responses are low-degree polynomials sent as evaluations.
 *   - Sec. 4.1.1: the prover's message is a huge sum in which every gate
 *     contributes to exactly one term; the message is a pass over the
 *     layer's gates, each gate's contribution computed independently and the
 *     contributions summed in F_p.
 *   - Sec. 2.2 / 4.1.2: the verifier's final "secret" is one value of the
 *     input's multilinear (low-degree) extension at a random point, computed
 *     in one pass over the input.
 *
 * The paper prints none of the formulas; the conventions below are the
 * standard GKR / sum-check definitions, fixed once:
 *   layers 0 = output ... d = input (the paper numbers them the other way);
 *   s_i = ceil(log2 S_i) (0 when S_i = 1), gate tables zero-padded to 2^s_i;
 *   eq(x,y) = xy + (1-x)(1-y), chi_x(r) = prod_k eq(bit_k(x), r_k);
 *   ~V(r) = sum_x chi_x(r) V[x]  (multilinear extension);
 *   f_i(a,b,c) = beta(z_i,a) [ add_i(a,b,c)(~V(b)+~V(c)) + mult_i(a,b,c)~V(b)~V(c) ]
 *   with add_i(a,b,c) = sum over ADD gates g of chi_g(a) chi_in1(b) chi_in2(c)
 *   (mult_i likewise), beta(z,a) = chi_a(z), and ~V the extension of layer
 *   i+1.  The sum-check runs over the s_i a-variables, then the s' = s_{i+1}
 *   b-variables, then the s' c-variables, least significant bit first.
 *   Transcript: msgs = V_0[0..S_0) | per layer: (G_j(0),G_j(1),G_j(2)) for
 *   every round j | v1 | v2 | h(2..s');  chals = z_0 | per layer: r_j for
 *   every round | tau.  h(t) = ~V_{i+1}(b* + t(c* - b*)); z_{i+1} and the
 *   next claim are that line and h at tau.
 *   Challenges: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) seeded with
 *   (seed << 8) | purpose, purpose 2 for GKR and 4 for the F2 sum-check; a
 *   field draw keeps the low 61 bits of an output and redraws on 2^61 - 1.
 *
 * Where a computation has a plain definition (circuit evaluation, the
 * multilinear extension, eq tables) it is that definition written out; the
 * prover's messages are computed gate by gate as Sec. 4.1.1 describes.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

#define P ((u64)0x1FFFFFFFFFFFFFFFULL) /* 2^61 - 1 */

/* ----------------------------------------------------------------- field */

static u64 f_red(u128 x) { return (u64)(x % P); }
static u64 f_add(u64 a, u64 b) { return f_red((u128)a + b); }
static u64 f_sub(u64 a, u64 b) { return f_red((u128)a + P - b); }
static u64 f_mul(u64 a, u64 b) { return f_red((u128)a * b); }
static u64 f_pow(u64 a, u64 e) {
    u64 r = 1;
    while (e) {
        if (e & 1) r = f_mul(r, a);
        a = f_mul(a, a);
        e >>= 1;
    }
    return r;
}
/* Fermat: a^(p-2) is the inverse of a != 0. */
static u64 f_inv(u64 a) { return f_pow(a, P - 2); }
/* eq(x, y) = x y + (1 - x)(1 - y) */
static u64 f_eq(u64 x, u64 y) { return f_add(f_mul(x, y), f_mul(f_sub(1, x), f_sub(1, y))); }

u64 or_field_add(u64 a, u64 b) { return f_add(a, b); }
u64 or_field_sub(u64 a, u64 b) { return f_sub(a, b); }
u64 or_field_mul(u64 a, u64 b) { return f_mul(a, b); }
u64 or_field_inv(u64 a) { return f_inv(a); }
u64 or_field_reduce_u128(u64 hi, u64 lo) { return f_red(((u128)hi << 64) | lo); }

/* ------------------------------------------------------------ splitmix64 */

typedef struct { u64 state; } sm64;
static void sm_init(sm64 *g, u64 seed, u64 purpose) { g->state = (seed << 8) | purpose; }
static u64 sm_next(sm64 *g) {
    g->state += 0x9E3779B97F4A7C15ULL;
    u64 z = g->state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static u64 sm_field(sm64 *g) {
    for (;;) {
        u64 x = sm_next(g) & P;
        if (x != P) return x;
    }
}

void or_splitmix_raw(u64 seed, u64 purpose, u64 n, u64 *out) {
    sm64 g; sm_init(&g, seed, purpose);
    for (u64 i = 0; i < n; i++) out[i] = sm_next(&g);
}
void or_splitmix_field(u64 seed, u64 purpose, u64 n, u64 *out) {
    sm64 g; sm_init(&g, seed, purpose);
    for (u64 i = 0; i < n; i++) out[i] = sm_field(&g);
}

/* -------------------------------------------------- threads (exact sums) */
/* Sec. 4.1.1: gate contributions are independent and summed in F_p; since
 * the sum is exact, splitting the gates into contiguous ranges and adding
 * the partial sums gives the same value for any thread count. */

typedef void (*range_fn)(void *ctx, u64 lo, u64 hi, u64 acc[3]);
typedef struct { range_fn fn; void *ctx; u64 lo, hi; u64 acc[3]; } job_t;
static void *job_run(void *p) { job_t *j = (job_t *)p; j->fn(j->ctx, j->lo, j->hi, j->acc); return NULL; }

static int g_threads = 1;
void or_set_threads(int t) { g_threads = t < 1 ? 1 : (t > 256 ? 256 : t); }

static void par_sum(u64 n, range_fn fn, void *ctx, u64 out[3]) {
    int T = g_threads;
    if ((u64)T > n / 4096 + 1) T = (int)(n / 4096 + 1);
    out[0] = out[1] = out[2] = 0;
    if (T <= 1) { fn(ctx, 0, n, out); return; }
    job_t jobs[256]; pthread_t th[256];
    for (int t = 0; t < T; t++) {
        jobs[t].fn = fn; jobs[t].ctx = ctx;
        jobs[t].lo = n * (u64)t / (u64)T; jobs[t].hi = n * (u64)(t + 1) / (u64)T;
        jobs[t].acc[0] = jobs[t].acc[1] = jobs[t].acc[2] = 0;
        pthread_create(&th[t], NULL, job_run, &jobs[t]);
    }
    for (int t = 0; t < T; t++) {
        pthread_join(th[t], NULL);
        for (int k = 0; k < 3; k++) out[k] = f_add(out[k], jobs[t].acc[k]);
    }
}

/* -------------------------------------------------------------- circuit */

typedef struct {
    u32 L;                 /* layers 0..L-1; layer L-1 is the input layer */
    const u32 *S;          /* S[i] = number of gates of layer i            */
    const uint8_t *const *type; /* [L-1] arrays: 0 = ADD, 1 = MUL          */
    const u32 *const *in1;      /* [L-1] arrays: wires into layer i+1      */
    const u32 *const *in2;
} circ_t;

static u32 log2ceil(u64 S) { u32 s = 0; while (((u64)1 << s) < S) s++; return s; }

u32 or_log2ceil(u64 S) { return log2ceil(S); }

/* 0 if the circuit is well formed: L >= 2, S[i] >= 1, types in {0,1},
 * every wire below 2^{s_{i+1}} (it may name a zero padding slot). */
int or_check_circuit(u32 L, const u32 *S, const uint8_t *const *type, const u32 *const *in1,
                     const u32 *const *in2) {
    if (L < 2) return -1;
    for (u32 i = 0; i < L; i++) if (S[i] == 0) return -1;
    for (u32 i = 0; i + 1 < L; i++) {
        u64 lim = (u64)1 << log2ceil(S[i + 1]);
        for (u32 g = 0; g < S[i]; g++) {
            if (type[i][g] > 1) return -1;
            if (in1[i][g] >= lim || in2[i][g] >= lim) return -1;
        }
    }
    return 0;
}

/* Transcript lengths (layout in the file header). */
void or_transcript_size(u32 L, const u32 *S, u64 *n_msgs, u64 *n_chals) {
    u64 m = S[0], c = log2ceil(S[0]);
    for (u32 i = 0; i + 1 < L; i++) {
        u64 s = log2ceil(S[i]), sp = log2ceil(S[i + 1]);
        u64 n = s + 2 * sp;
        m += 3 * n + 2 + (sp >= 2 ? sp - 1 : 0);
        c += n + 1;
    }
    *n_msgs = m; *n_chals = c;
}

/* Circuit evaluation, layer d-1 down to 0: V_i[g] = V_{i+1}[in1] op V_{i+1}[in2].
 * V[i] has 2^{s_i} entries; the padding beyond S[i] is zero. */
static void evaluate(const circ_t *c, const u64 *inputs, u64 **V) {
    u32 d = c->L - 1;
    u64 n = (u64)1 << log2ceil(c->S[d]);
    memset(V[d], 0, n * sizeof(u64));
    memcpy(V[d], inputs, c->S[d] * sizeof(u64));
    for (int i = (int)d - 1; i >= 0; i--) {
        u64 np = (u64)1 << log2ceil(c->S[i]);
        memset(V[i], 0, np * sizeof(u64));
        for (u32 g = 0; g < c->S[i]; g++) {
            u64 x = V[i + 1][c->in1[i][g]], y = V[i + 1][c->in2[i][g]];
            V[i][g] = c->type[i][g] == 0 ? f_add(x, y) : f_mul(x, y);
        }
    }
}

int or_evaluate(u32 L, const u32 *S, const uint8_t *const *type, const u32 *const *in1,
                const u32 *const *in2, const u64 *inputs, u64 *const *V) {
    circ_t c = {L, S, type, in1, in2};
    if (or_check_circuit(L, S, type, in1, in2)) return -1;
    evaluate(&c, inputs, (u64 **)V);
    return 0;
}

/* ---------------------------------------------- multilinear extensions */

/* One variable of a multilinear extension, least significant bit first:
 * ~T(r, rest) = (1 - r) ~T(0, rest) + r ~T(1, rest), so binding the lowest
 * variable to r maps T[2m], T[2m+1] to T[2m] + r (T[2m+1] - T[2m]). */
static void fold(u64 *T, u64 half, u64 r) {
    for (u64 m = 0; m < half; m++) T[m] = f_add(T[2 * m], f_mul(r, f_sub(T[2 * m + 1], T[2 * m])));
}

/* ~T(pt) for a table of 2^s entries, by binding the variables one by one. */
static u64 mle(const u64 *T, u32 s, const u64 *pt) {
    u64 n = (u64)1 << s;
    u64 *W = (u64 *)malloc(n * sizeof(u64));
    memcpy(W, T, n * sizeof(u64));
    for (u32 k = 0; k < s; k++) fold(W, n >> (k + 1), pt[k]);
    u64 v = W[0];
    free(W);
    return v;
}
u64 or_mle(const u64 *T, u32 s, const u64 *pt) { return mle(T, s, pt); }

/* eq table E[x] = chi_x(pt) for x < 2^s, built coordinate by coordinate:
 * chi over k+1 coordinates = chi over the first k times eq(bit_k, pt_k). */
static void eq_table(const u64 *pt, u32 s, u64 *E) {
    E[0] = 1;
    for (u32 k = 0; k < s; k++) {
        u64 h = (u64)1 << k;
        for (u64 x = 0; x < h; x++) {
            u64 e = E[x];
            E[x] = f_mul(e, f_sub(1, pt[k]));
            E[x + h] = f_mul(e, pt[k]);
        }
    }
}
void or_eq_table(const u64 *pt, u32 s, u64 *E) { eq_table(pt, s, E); }

/* Lagrange interpolation of the values y[0..D] at the nodes 0..D, at x. */
static u64 lagrange(const u64 *y, u32 D, u64 x) {
    u64 acc = 0;
    for (u32 i = 0; i <= D; i++) {
        u64 num = 1, den = 1;
        for (u32 j = 0; j <= D; j++) {
            if (j == i) continue;
            num = f_mul(num, f_sub(x, j));
            den = f_mul(den, f_sub(i, j));
        }
        acc = f_add(acc, f_mul(y[i], f_mul(num, f_inv(den))));
    }
    return acc;
}
u64 or_lagrange(const u64 *y, u32 D, u64 x) { return lagrange(y, D, x); }

/* ------------------------------------------------ per-gate prover rounds */

/* State of one sum-check round over layer i, shared by the workers. */
typedef struct {
    const circ_t *c;
    u32 i, s, sp;
    u32 j;             /* round, 0 .. s + 2 sp - 1 */
    const u64 *Vn;     /* V_{i+1} (Boolean-point values) */
    const u64 *chi;    /* per gate: chi of the gate's coordinates over the bound prefix */
    const u64 *z;      /* z_i */
    u64 betaC;         /* prod_{k<j} eq(z_k, r_k) during the a-variables */
    const u64 *Bsuf;   /* a-variables: Bsuf[m] = prod_{k>j} eq(z_k, bit of m)  */
    u64 betaA;         /* beta(z, a*) once the a-variables are bound */
    const u64 *Fb;     /* V_{i+1} with the bound b-variables folded in */
    const u64 *Fc;     /* V_{i+1} with the bound c-variables folded in */
    u64 v1;            /* ~V_{i+1}(b*) during the c-variables */
    u64 r;             /* challenge applied by upd_range */
    u64 *chi_out;
} round_t;

/* The gate's coordinate that round j binds, and the value of the gate's
 * wiring term op(~V(b-part), ~V(c-part)) at t for the point
 * (r_<j, t, gate's own bits beyond j). */
static u64 gate_bit(const round_t *R, u64 g) {
    if (R->j < R->s) return (g >> R->j) & 1;
    if (R->j < R->s + R->sp) return (R->c->in1[R->i][g] >> (R->j - R->s)) & 1;
    return (R->c->in2[R->i][g] >> (R->j - R->s - R->sp)) & 1;
}

/* ~V at a point whose first k coordinates are folded into F, coordinate k is
 * t and the rest are the bits of idx above k: multilinear in coordinate k. */
static u64 partial_value(const u64 *F, u32 k, u64 idx, u64 t) {
    u64 m = idx >> (k + 1);
    u64 lo = F[2 * m], hi = F[2 * m + 1];
    return f_add(f_mul(f_sub(1, t), lo), f_mul(t, hi));
}

static void terms_range(void *ctx, u64 lo, u64 hi, u64 acc[3]) {
    const round_t *R = (const round_t *)ctx;
    const circ_t *c = R->c;
    u32 i = R->i;
    for (u64 g = lo; g < hi; g++) {
        u64 bit = gate_bit(R, g);
        u64 a1 = c->in1[i][g], a2 = c->in2[i][g];
        for (u64 t = 0; t < 3; t++) {
            u64 e = f_eq(bit, t); /* the gate's own coordinate at the current variable */
            if (e == 0) continue;
            u64 beta, vb, vc;
            if (R->j < R->s) {
                /* a-variable: beta(z, (r_<j, t, g_>j)); b and c are the Boolean wires. */
                beta = f_mul(f_mul(R->betaC, f_eq(R->z[R->j], t)), R->Bsuf[g >> (R->j + 1)]);
                vb = R->Vn[a1];
                vc = R->Vn[a2];
            } else if (R->j < R->s + R->sp) {
                beta = R->betaA;
                vb = partial_value(R->Fb, R->j - R->s, a1, t);
                vc = R->Vn[a2];
            } else {
                beta = R->betaA;
                vb = R->v1;
                vc = partial_value(R->Fc, R->j - R->s - R->sp, a2, t);
            }
            u64 w = c->type[i][g] == 0 ? f_add(vb, vc) : f_mul(vb, vc);
            u64 term = f_mul(f_mul(R->chi[g], e), f_mul(beta, w));
            acc[t] = f_add(acc[t], term);
        }
    }
}

/* suffix of beta: Bsuf[m] = prod_{k=j+1}^{s-1} eq(z_k, bit_{k-j-1}(m)) */
static void bsuf_range(void *ctx, u64 lo, u64 hi, u64 acc[3]) {
    const round_t *R = (const round_t *)ctx;
    (void)acc;
    u64 *B = (u64 *)R->Bsuf;
    for (u64 m = lo; m < hi; m++) {
        u64 b = 1;
        for (u32 k = R->j + 1; k < R->s; k++) b = f_mul(b, f_eq(R->z[k], (m >> (k - R->j - 1)) & 1));
        B[m] = b;
    }
}

static void upd_range(void *ctx, u64 lo, u64 hi, u64 acc[3]) {
    const round_t *R = (const round_t *)ctx;
    (void)acc;
    for (u64 g = lo; g < hi; g++) R->chi_out[g] = f_mul(R->chi[g], f_eq(gate_bit(R, g), R->r));
}

/* Prove one circuit.  msgs / chals must hold or_transcript_size() entries. */
int or_prove(u32 L, const u32 *S, const uint8_t *const *type, const u32 *const *in1,
             const u32 *const *in2, const u64 *inputs, u64 seed, u64 *msgs, u64 *chals) {
    if (or_check_circuit(L, S, type, in1, in2)) return -1;
    for (u32 g = 0; g < S[L - 1]; g++) if (inputs[g] >= P) return -2;
    circ_t c = {L, S, type, in1, in2};
    u32 d = L - 1;
    u64 **V = (u64 **)malloc(L * sizeof(u64 *));
    u32 smax = 0;
    u64 gmax = 0;
    for (u32 i = 0; i < L; i++) {
        u32 s = log2ceil(S[i]);
        if (s > smax) smax = s;
        if (S[i] > gmax) gmax = S[i];
        V[i] = (u64 *)malloc(((u64)1 << s) * sizeof(u64));
    }
    evaluate(&c, inputs, V);

    sm64 rng; sm_init(&rng, seed, 2);
    u64 mi = 0, ci = 0;
    for (u32 g = 0; g < S[0]; g++) msgs[mi++] = V[0][g];

    u64 *z = (u64 *)calloc(smax + 1, sizeof(u64));
    u64 *r = (u64 *)calloc(3 * (u64)smax + 1, sizeof(u64));
    u32 s0 = log2ceil(S[0]);
    for (u32 k = 0; k < s0; k++) { z[k] = sm_field(&rng); chals[ci++] = z[k]; }

    u64 *chi = (u64 *)malloc(gmax * sizeof(u64));
    u64 *chi2 = (u64 *)malloc(gmax * sizeof(u64));
    u64 *Bsuf = (u64 *)malloc(((u64)1 << smax) * sizeof(u64) + 8);
    u64 *Fb = (u64 *)malloc(((u64)1 << smax) * sizeof(u64));
    u64 *Fc = (u64 *)malloc(((u64)1 << smax) * sizeof(u64));
    u64 *bstar = (u64 *)calloc(smax + 1, sizeof(u64));
    u64 *cstar = (u64 *)calloc(smax + 1, sizeof(u64));
    u64 *lt = (u64 *)calloc(smax + 1, sizeof(u64));

    for (u32 i = 0; i < d; i++) {
        u32 s = log2ceil(S[i]), sp = log2ceil(S[i + 1]);
        u32 n = s + 2 * sp;
        u64 np = (u64)1 << sp;
        for (u64 g = 0; g < S[i]; g++) chi[g] = 1;
        memcpy(Fb, V[i + 1], np * sizeof(u64));
        memcpy(Fc, V[i + 1], np * sizeof(u64));
        round_t R;
        memset(&R, 0, sizeof R);
        R.c = &c; R.i = i; R.s = s; R.sp = sp; R.Vn = V[i + 1]; R.z = z;
        /* beta over zero a-coordinates is 1; otherwise set once a* is bound */
        R.betaC = 1; R.betaA = 1; R.Fb = Fb; R.Fc = Fc; R.Bsuf = Bsuf;
        for (u32 j = 0; j < n; j++) {
            R.j = j; R.chi = chi;
            if (j < s) {
                u64 dummy[3];
                par_sum((u64)1 << (s - j - 1), bsuf_range, &R, dummy);
            }
            if (j == s + sp) R.v1 = Fb[0];
            u64 G[3];
            par_sum(S[i], terms_range, &R, G);
            msgs[mi++] = G[0]; msgs[mi++] = G[1]; msgs[mi++] = G[2];
            /* the challenge is drawn only after the message is complete */
            r[j] = sm_field(&rng);
            chals[ci++] = r[j];
            R.r = r[j]; R.chi_out = chi2;
            par_sum(S[i], upd_range, &R, G);
            u64 *tmp = chi; chi = chi2; chi2 = tmp;
            if (j < s) {
                R.betaC = f_mul(R.betaC, f_eq(z[j], r[j]));
                if (j == s - 1) R.betaA = R.betaC;
            } else if (j < s + sp) {
                fold(Fb, np >> (j - s + 1), r[j]);
            } else {
                fold(Fc, np >> (j - s - sp + 1), r[j]);
            }
        }
        /* v1 = ~V_{i+1}(b*), v2 = ~V_{i+1}(c*): the fully folded tables. */
        u64 v1 = Fb[0], v2 = Fc[0];
        msgs[mi++] = v1; msgs[mi++] = v2;
        for (u32 k = 0; k < sp; k++) { bstar[k] = r[s + k]; cstar[k] = r[s + sp + k]; }
        /* h(t) = ~V_{i+1}(l(t)), l(t) = b* + t (c* - b*), for t = 2 .. sp */
        for (u64 t = 2; t <= sp; t++) {
            for (u32 k = 0; k < sp; k++) lt[k] = f_add(bstar[k], f_mul(t, f_sub(cstar[k], bstar[k])));
            msgs[mi++] = mle(V[i + 1], sp, lt);
        }
        u64 tau = sm_field(&rng);
        chals[ci++] = tau;
        for (u32 k = 0; k < sp; k++) z[k] = f_add(bstar[k], f_mul(tau, f_sub(cstar[k], bstar[k])));
    }

    for (u32 i = 0; i < L; i++) free(V[i]);
    free(V); free(z); free(r); free(chi); free(chi2); free(Bsuf); free(Fb); free(Fc);
    free(bstar); free(cstar); free(lt);
    return 0;
}

/* ------------------------------------------------------------- verifier */

typedef struct { const circ_t *c; u32 i; const u64 *Ea, *Eb, *Ec; } wire_t;

/* add~(a*,b*,c*) into acc[0], mult~(a*,b*,c*) into acc[1]: a sum over the
 * layer's gates of chi_g(a*) chi_in1(b*) chi_in2(c*). */
static void wiring_range(void *ctx, u64 lo, u64 hi, u64 acc[3]) {
    const wire_t *W = (const wire_t *)ctx;
    for (u64 g = lo; g < hi; g++) {
        u64 v = f_mul(W->Ea[g], f_mul(W->Eb[W->c->in1[W->i][g]], W->Ec[W->c->in2[W->i][g]]));
        u32 t = W->c->type[W->i][g];
        acc[t] = f_add(acc[t], v);
    }
}

/* Verify a GKR transcript.  Returns 0 with *accepted set, or <0 on a
 * malformed circuit / input.  On rejection *why_layer, *why_round and
 * *why_check say where: check 1 = malformed transcript (length or a value
 * not below p), 2 = round sum G(0)+G(1) != claim, 3 = final wiring identity,
 * 4 = line endpoints (v1 != v2 when layer i+1 has one gate), 5 = the claim
 * about the input layer differs from the input's multilinear extension. */
int or_verify(u32 L, const u32 *S, const uint8_t *const *type, const u32 *const *in1,
              const u32 *const *in2, const u64 *inputs, u64 seed, const u64 *msgs, u64 n_msgs,
              int *accepted, int *why_layer, int *why_round, int *why_check) {
    if (or_check_circuit(L, S, type, in1, in2)) return -1;
    for (u32 g = 0; g < S[L - 1]; g++) if (inputs[g] >= P) return -2;
    circ_t c = {L, S, type, in1, in2};
    u32 d = L - 1;
    *accepted = 0; *why_layer = -1; *why_round = -1; *why_check = 0;
    u64 want_m, want_c;
    or_transcript_size(L, S, &want_m, &want_c);
    if (n_msgs != want_m) { *why_check = 1; return 0; }
    for (u64 k = 0; k < n_msgs; k++) if (msgs[k] >= P) { *why_check = 1; return 0; }

    u32 smax = 0;
    u64 gmax = 0;
    for (u32 i = 0; i < L; i++) {
        if (log2ceil(S[i]) > smax) smax = log2ceil(S[i]);
        if (S[i] > gmax) gmax = S[i];
    }
    u64 tmax = (u64)1 << smax;
    u64 *T = (u64 *)calloc(tmax, sizeof(u64));
    u64 *Ea = (u64 *)malloc(tmax * sizeof(u64));
    u64 *Eb = (u64 *)malloc(tmax * sizeof(u64));
    u64 *Ec = (u64 *)malloc(tmax * sizeof(u64));
    u64 *z = (u64 *)calloc(smax + 1, sizeof(u64));
    u64 *r = (u64 *)calloc(3 * (u64)smax + 1, sizeof(u64));
    u64 *y = (u64 *)calloc(smax + 2, sizeof(u64));

    sm64 rng; sm_init(&rng, seed, 2);
    u64 mi = 0;
    u32 s0 = log2ceil(S[0]);
    memset(T, 0, ((u64)1 << s0) * sizeof(u64));
    for (u32 g = 0; g < S[0]; g++) T[g] = msgs[mi++];
    for (u32 k = 0; k < s0; k++) z[k] = sm_field(&rng);
    u64 claim = mle(T, s0, z);
    int ok = 1;

    for (u32 i = 0; i < d && ok; i++) {
        u32 s = log2ceil(S[i]), sp = log2ceil(S[i + 1]);
        u32 n = s + 2 * sp;
        for (u32 j = 0; j < n; j++) {
            const u64 *G = msgs + mi;
            mi += 3;
            if (f_add(G[0], G[1]) != claim) {
                *why_layer = (int)i; *why_round = (int)j; *why_check = 2; ok = 0; break;
            }
            r[j] = sm_field(&rng);
            claim = lagrange(G, 2, r[j]);
        }
        if (!ok) break;
        u64 v1 = msgs[mi++], v2 = msgs[mi++];
        /* final check of the layer: claim = beta(z, a*) [add~ (v1+v2) + mult~ v1 v2] */
        u64 beta = 1;
        for (u32 k = 0; k < s; k++) beta = f_mul(beta, f_eq(z[k], r[k]));
        eq_table(r, s, Ea);
        eq_table(r + s, sp, Eb);
        eq_table(r + s + sp, sp, Ec);
        wire_t W = {&c, i, Ea, Eb, Ec};
        u64 am[3];
        par_sum(S[i], wiring_range, &W, am);
        u64 rhs = f_mul(beta, f_add(f_mul(am[0], f_add(v1, v2)), f_mul(am[1], f_mul(v1, v2))));
        if (rhs != claim) { *why_layer = (int)i; *why_round = (int)n; *why_check = 3; ok = 0; break; }
        if (sp == 0 && v1 != v2) { *why_layer = (int)i; *why_check = 4; ok = 0; break; }
        /* the line polynomial h, degree <= sp, given at t = 0 .. max(sp, 1) */
        u32 D = sp > 1 ? sp : 1;
        y[0] = v1; y[1] = v2;
        for (u32 t = 2; t <= sp; t++) y[t] = msgs[mi++];
        u64 tau = sm_field(&rng);
        claim = lagrange(y, D, tau);
        for (u32 k = 0; k < sp; k++) z[k] = f_add(r[s + k], f_mul(tau, f_sub(r[s + sp + k], r[s + k])));
    }
    if (ok) {
        /* the verifier's own secret: the input's multilinear extension at z_d */
        u32 sd = log2ceil(S[d]);
        memset(T, 0, ((u64)1 << sd) * sizeof(u64));
        memcpy(T, inputs, S[d] * sizeof(u64));
        if (mle(T, sd, z) != claim) { *why_layer = (int)d; *why_check = 5; ok = 0; }
    }
    *accepted = ok;
    free(T); free(Ea); free(Eb); free(Ec); free(z); free(r); free(y);
    return 0;
}

/* ------------------------------------------------------ F2 sum-check */

typedef struct { const u64 *A; } sq_t;
/* G(t) = sum_m ((1-t) A[2m] + t A[2m+1])^2 at t = 0, 1, 2 */
static void sq_range(void *ctx, u64 lo, u64 hi, u64 acc[3]) {
    const u64 *A = ((const sq_t *)ctx)->A;
    for (u64 m = lo; m < hi; m++) {
        u64 a0 = A[2 * m], a1 = A[2 * m + 1];
        u64 a2 = f_sub(f_add(a1, a1), a0);
        acc[0] = f_add(acc[0], f_mul(a0, a0));
        acc[1] = f_add(acc[1], f_mul(a1, a1));
        acc[2] = f_add(acc[2], f_mul(a2, a2));
    }
}

static int is_pow2(u64 n) { return n && !(n & (n - 1)); }

/* Sum-check for F2 = sum_x a(x)^2 over {0,1}^l, n = 2^l:
 * msgs = [F2, G_1(0), G_1(1), G_1(2), ..., G_l(2)], chals = r_1 .. r_l. */
int or_f2sc_prove(const u32 *freq, u64 n, u64 seed, u64 *msgs, u64 *chals) {
    if (!is_pow2(n)) return -1;
    u32 l = log2ceil(n);
    u64 *A = (u64 *)malloc(n * sizeof(u64));
    for (u64 x = 0; x < n; x++) A[x] = freq[x];
    u64 F2 = 0;
    for (u64 x = 0; x < n; x++) F2 = f_add(F2, f_mul(A[x], A[x]));
    msgs[0] = F2;
    sm64 rng; sm_init(&rng, seed, 4);
    for (u32 j = 0; j < l; j++) {
        sq_t ctx = {A};
        u64 G[3];
        par_sum(n >> (j + 1), sq_range, &ctx, G);
        msgs[1 + 3 * j] = G[0]; msgs[2 + 3 * j] = G[1]; msgs[3 + 3 * j] = G[2];
        u64 rj = sm_field(&rng);
        chals[j] = rj;
        fold(A, n >> (j + 1), rj);
    }
    free(A);
    return 0;
}

int or_f2sc_verify(const u32 *freq, u64 n, u64 seed, const u64 *msgs, u64 n_msgs, int *accepted,
                   int *why_round, int *why_check) {
    if (!is_pow2(n)) return -1;
    u32 l = log2ceil(n);
    *accepted = 0; *why_round = -1; *why_check = 0;
    if (n_msgs != 1 + 3 * (u64)l) { *why_check = 1; return 0; }
    for (u64 k = 0; k < n_msgs; k++) if (msgs[k] >= P) { *why_check = 1; return 0; }
    sm64 rng; sm_init(&rng, seed, 4);
    u64 claim = msgs[0];
    u64 *r = (u64 *)calloc(l + 1, sizeof(u64));
    for (u32 j = 0; j < l; j++) {
        const u64 *G = msgs + 1 + 3 * j;
        if (f_add(G[0], G[1]) != claim) { *why_round = (int)j; *why_check = 2; free(r); return 0; }
        r[j] = sm_field(&rng);
        claim = lagrange(G, 2, r[j]);
    }
    u64 *A = (u64 *)malloc(n * sizeof(u64));
    for (u64 x = 0; x < n; x++) A[x] = freq[x];
    u64 ar = mle(A, l, r);
    free(A); free(r);
    if (f_mul(ar, ar) != claim) { *why_check = 5; return 0; }
    *accepted = 1;
    return 0;
}

/* ------------------------------------- non-interactive F2 (Sec. 3.2)
 *
 * The reading fixed for this build (the paper gives the protocol's outline
 * only): the universe [n] is a v x h grid, v = ceil(n / h), cell (row y,
 * column j) holding a_i for i = j v + y (zero for i >= n).  h divides
 * (p - 1) / 2, so F_p has subgroups H of order h and G of order 2h, with
 * generators w_h = g^((p-1)/h) and xi = g^((p-1)/(2h)), g = 37 a primitive
 * root; xi^2 = w_h.  Row y is the polynomial f_y of degree < h with
 * f_y(w_h^j) = a(j, y).  The proof is g(X) = sum_y f_y(X)^2 (degree
 * <= 2h - 2) at the 2h points xi^k: even k are the data squared, odd k need
 * f_y at the coset xi H.  The verifier's secret r (seed, purpose 9) gives
 * f_y(r) for each row (v words while streaming); it accepts iff
 * g(r) = sum_y f_y(r)^2, and F2 = sum_j g(w_h^j) = sum_j msgs[2j]. */

#define NIF2_ROOT 37
#define NIF2_PURPOSE 9

static u64 nif2_root(u64 N) { return ((P - 1) % N) ? 0 : f_pow(NIF2_ROOT, (P - 1) / N); }
u64 or_nif2_root(u64 N) { return nif2_root(N); }

/* Lagrange basis of the subgroup {w^0, .., w^(N-1)} at x:
 * L_j(x) = w^j (x^N - 1) / (N (x - w^j)); at x = w^m it is [j == m]. */
static void subgroup_basis(u64 w, u64 N, u64 x, u64 *L) {
    u64 xN = f_pow(x, N), wj = 1, hit = N;
    for (u64 j = 0; j < N; j++, wj = f_mul(wj, w))
        if (wj == x) hit = j;
    if (hit < N) {
        for (u64 j = 0; j < N; j++) L[j] = j == hit;
        return;
    }
    wj = 1;
    for (u64 j = 0; j < N; j++, wj = f_mul(wj, w))
        L[j] = f_mul(f_mul(wj, f_sub(xN, 1)), f_inv(f_mul(N % P, f_sub(x, wj))));
}

static u64 cell(const u64 *a, u64 n, u64 v, u64 j, u64 y) {
    const u64 i = j * v + y;
    return i < n ? a[i] % P : 0;
}

typedef struct { const u64 *a; u64 n, h, v, xi; u64 *msgs; int t, T; } nif2_job;

/* Odd message points k = 2m + 1, m = t, t + T, ...: f_y(xi^k) by the
 * Lagrange formula, squared and summed over the rows. */
static void *nif2_odd(void *p) {
    nif2_job *J = (nif2_job *)p;
    const u64 h = J->h, wh = nif2_root(h);
    u64 *L = (u64 *)malloc(h * sizeof(u64));
    for (u64 m = (u64)J->t; m < h; m += (u64)J->T) {
        const u64 k = 2 * m + 1;
        subgroup_basis(wh, h, f_pow(J->xi, k), L);
        u64 g = 0;
        for (u64 y = 0; y < J->v; y++) {
            u64 fy = 0;
            for (u64 j = 0; j < h; j++) fy = f_add(fy, f_mul(cell(J->a, J->n, J->v, j, y), L[j]));
            g = f_add(g, f_mul(fy, fy));
        }
        J->msgs[k] = g;
    }
    free(L);
    return NULL;
}

/* msgs[0 .. 2h): g(xi^k).  Returns -1 if h does not divide (p - 1) / 2. */
int or_nif2_prove(const u64 *a, u64 n, u64 h, u64 *msgs) {
    if (h < 1 || h % 2 == 0 || ((P - 1) / 2) % h) return -1;
    const u64 v = (n + h - 1) / h, xi = nif2_root(2 * h);
    for (u64 j = 0; j < h; j++) {  /* even points: the data */
        u64 g = 0;
        for (u64 y = 0; y < v; y++) g = f_add(g, f_mul(cell(a, n, v, j, y), cell(a, n, v, j, y)));
        msgs[2 * j] = g;
    }
    int T = g_threads < 1 ? 1 : g_threads;
    pthread_t th[256];
    nif2_job jobs[256];
    for (int t = 0; t < T; t++) {
        jobs[t] = (nif2_job){a, n, h, v, xi, msgs, t, T};
        pthread_create(&th[t], NULL, nif2_odd, &jobs[t]);
    }
    for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
    return 0;
}

/* The verifier: r from (seed, purpose 9); accepted iff g(r) (interpolated
 * from the 2h points) equals sum_y f_y(r)^2.  f2 = sum_j msgs[2j]. */
int or_nif2_verify(const u64 *a, u64 n, u64 h, u64 seed, const u64 *msgs, u64 n_msgs, int *accepted,
                   u64 *f2) {
    if (h < 1 || h % 2 == 0 || ((P - 1) / 2) % h) return -1;
    *accepted = 0;
    *f2 = 0;
    if (n_msgs != 2 * h) return 0;
    for (u64 k = 0; k < n_msgs; k++) if (msgs[k] >= P) return 0;
    const u64 v = (n + h - 1) / h;
    sm64 rng; sm_init(&rng, seed, NIF2_PURPOSE);
    const u64 r = sm_field(&rng);
    u64 *L = (u64 *)malloc(2 * h * sizeof(u64));
    subgroup_basis(nif2_root(h), h, r, L);
    u64 rhs = 0;
    for (u64 y = 0; y < v; y++) {
        u64 fy = 0;
        for (u64 j = 0; j < h; j++) fy = f_add(fy, f_mul(cell(a, n, v, j, y), L[j]));
        rhs = f_add(rhs, f_mul(fy, fy));
    }
    subgroup_basis(nif2_root(2 * h), 2 * h, r, L);
    u64 gr = 0;
    for (u64 k = 0; k < 2 * h; k++) gr = f_add(gr, f_mul(msgs[k], L[k]));
    free(L);
    for (u64 j = 0; j < h; j++) *f2 = f_add(*f2, msgs[2 * j]);
    *accepted = gr == rhs;
    return 0;
}
