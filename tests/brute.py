"""Brute-force definitions in pure Python integers, for tiny inputs only.

These evaluate the objects of the GKR protocol straight from their
definitions (no folding, no per-gate bookkeeping), to pin the oracle:
  chi_x(r) = prod_k eq(bit_k(x), r_k),  eq(x, y) = xy + (1-x)(1-y)
  ~V(r)    = sum over all Boolean x of chi_x(r) V[x]
  f_i(a,b,c) = beta(z,a) sum_g chi_g(a) chi_in1(b) chi_in2(c) op_g(~V(b), ~V(c))
  G_j(t)   = sum over Boolean x_{>j} of f_i(r_<j, t, x_{>j})
"""
import itertools

P = (1 << 61) - 1


def eq(x, y):
    return (x * y + (1 - x) * (1 - y)) % P


def chi(x, r):
    out = 1
    for k, rk in enumerate(r):
        out = out * eq((x >> k) & 1, rk) % P
    return out


def mle(T, r):
    return sum(chi(x, r) * int(T[x]) for x in range(len(T))) % P


def log2ceil(n):
    s = 0
    while (1 << s) < n:
        s += 1
    return s


def evaluate(circ, inputs):
    """Gate values by definition, padded to powers of two."""
    d = len(circ.sizes) - 1
    V = [None] * (d + 1)
    V[d] = [int(v) for v in inputs] + [0] * ((1 << log2ceil(circ.sizes[d])) - circ.sizes[d])
    for i in range(d - 1, -1, -1):
        row = []
        for g in range(circ.sizes[i]):
            x, y = V[i + 1][int(circ.in1[i][g])], V[i + 1][int(circ.in2[i][g])]
            row.append((x + y) % P if circ.types[i][g] == 0 else x * y % P)
        V[i] = row + [0] * ((1 << log2ceil(circ.sizes[i])) - circ.sizes[i])
    return V


def layer_f(circ, V, i, z, a, b, c):
    """f_i at an arbitrary point (a, b, c)."""
    beta = 1
    for zk, ak in zip(z, a):
        beta = beta * eq(zk, ak) % P
    vb, vc = mle(V[i + 1], b), mle(V[i + 1], c)
    acc = 0
    for g in range(circ.sizes[i]):
        w = chi(g, a) * chi(int(circ.in1[i][g]), b) % P * chi(int(circ.in2[i][g]), c) % P
        op = (vb + vc) % P if circ.types[i][g] == 0 else vb * vc % P
        acc = (acc + w * op) % P
    return beta * acc % P


def round_message(circ, V, i, z, r_prefix, t):
    """G_j(t), j = len(r_prefix), summing f_i over the remaining Boolean variables."""
    s, sp = log2ceil(circ.sizes[i]), log2ceil(circ.sizes[i + 1])
    n = s + 2 * sp
    j = len(r_prefix)
    acc = 0
    for tail in itertools.product((0, 1), repeat=n - j - 1):
        pt = list(r_prefix) + [t] + list(tail)
        acc = (acc + layer_f(circ, V, i, z, pt[:s], pt[s:s + sp], pt[s + sp:])) % P
    return acc


def layer_sum(circ, V, i, z):
    """sum over the whole hypercube of f_i; equals ~V_i(z)."""
    s, sp = log2ceil(circ.sizes[i]), log2ceil(circ.sizes[i + 1])
    acc = 0
    for pt in itertools.product((0, 1), repeat=s + 2 * sp):
        acc = (acc + layer_f(circ, V, i, z, pt[:s], pt[s:s + sp], pt[s + sp:])) % P
    return acc


def transcript_by_definition(circ, inputs, chals):
    """The whole GKR transcript from the definitions, given the challenge
    sequence (z_0 | per layer r_1..r_n, tau)."""
    V = evaluate(circ, inputs)
    d = len(circ.sizes) - 1
    msgs = [V[0][g] for g in range(circ.sizes[0])]
    ci = 0
    s0 = log2ceil(circ.sizes[0])
    z = [int(c) for c in chals[ci:ci + s0]]
    ci += s0
    for i in range(d):
        s, sp = log2ceil(circ.sizes[i]), log2ceil(circ.sizes[i + 1])
        n = s + 2 * sp
        r = []
        for j in range(n):
            for t in (0, 1, 2):
                msgs.append(round_message(circ, V, i, z, r, t))
            r.append(int(chals[ci]))
            ci += 1
        bstar, cstar = r[s:s + sp], r[s + sp:]
        msgs.append(mle(V[i + 1], bstar))
        msgs.append(mle(V[i + 1], cstar))
        for t in range(2, sp + 1):
            msgs.append(mle(V[i + 1], [(b + t * (c - b)) % P for b, c in zip(bstar, cstar)]))
        tau = int(chals[ci])
        ci += 1
        z = [(b + tau * (c - b)) % P for b, c in zip(bstar, cstar)]
    return msgs


def f2sc_by_definition(a, chals):
    """Sum-check transcript of sum_x ~a(x)^2 from the definition."""
    l = log2ceil(len(a))
    msgs = [sum(int(v) ** 2 for v in a) % P]
    for j in range(l):
        for t in (0, 1, 2):
            acc = 0
            for tail in itertools.product((0, 1), repeat=l - j - 1):
                pt = [int(c) for c in chals[:j]] + [t] + list(tail)
                acc = (acc + mle(a, pt) ** 2) % P
            msgs.append(acc)
    return msgs


def splitmix64(seed, purpose, n):
    """Reference SplitMix64 in Python integers (public algorithm)."""
    M = (1 << 64) - 1
    st = ((seed << 8) | purpose) & M
    out = []
    for _ in range(n):
        st = (st + 0x9E3779B97F4A7C15) & M
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        out.append(z ^ (z >> 31))
    return out
