#!/usr/bin/env python3
"""Generate straight-line HIP code for the cell-body multipole expansion.

The paper produces its interaction routines up to p = 8 by metaprogramming
(Multipole Error Bounds section: translating a computer-algebra
representation directly into C). This build step does the same for the GPU:
for every order p it emits fully unrolled code, with no loops and no arrays,
so that every intermediate lives in a register.

Derivatives of the softened Green's function G(R) = -(|R|^2 + e^2)^(-1/2)
are built with the Hermite recursion of McMurchie and Davidson for radial
functions f(s), s = |R|^2 + e^2:
    R^(n)_000 = F_n = 2^n f^(n)(s) = (-1)^(n+1) (2n-1)!! s^(-n-1/2),
    R^(n)_{..,k+1,..} = k R^(n+1)_{..,k-1,..} + x_k R^(n+1)_{..,k,..},
    d^alpha G = R^(0)_alpha.
The recursion is used along z and y; along x the closed form
    R^(0)_{t,u,v} = sum_j t! / (j! (t-2j)! 2^j) X^(t-2j) R^(t-j)_{0,u,v}
replaces the last triangle of the recursion (fewer operations when only
n = 0 is needed).

Emitted functions (T is float or double):
  expansion_fwd<P,T,POT>(X,Y,Z,e2,M,ax,ay,az,ph)
      ax += sum_alpha M[alpha] d^(alpha+e_x) G (likewise y, z); ph += sum M d^alpha G
  expansion_sink_adj<P,T>(X,Y,Z,e2,M,bx,by,bz,gx,gy,gz)
      g_l += sum_k b_k sum_alpha M[alpha] d^(alpha+e_k+e_l) G
  expansion_cell_adj<P,T>(X,Y,Z,e2,bx,by,bz,row)
      row[alpha] += sum_k b_k d^(alpha+e_k) G   (row: registers of the lane)
M holds the (weighted, scaled) moments in slot order: by order, then x
exponent descending, then y exponent descending.
"""
import math
import os
import sys

PMAX = 8


def slot(a, b, c):
    n = a + b + c
    return n * (n + 1) * (n + 2) // 6 + (b + c) * (b + c + 1) // 2 + c


def lit(x):
    return f"T({float(x)!r})"


class Emitter:
    def __init__(self, K, row_barriers=False):
        self.K = K
        self.lines = []
        # scheduling barriers between z-rows keep the operands (moments) of each
        # row from being loaded all at once at the top: fewer live registers
        self.row_barriers = row_barriers

    def e(self, s):
        self.lines.append("  " + s)

    def radial(self):
        """F_n = 2^n f^(n)(s), n <= K, for both softening kernels. Plummer:
        s = |R|^2 + e2, f = -s^(-1/2). K1 (e2 the squared kernel radius):
        outside (s = |R|^2 >= e2) the Newtonian f = -s^(-1/2); inside f is the
        quartic -Q(v) / (256 eps) in v = 1 - s / e2, so F_n = -(-2)^n Q^(n)(v) /
        (256 eps^(2n+1)): Q(v) = 256 + 128 v + 96 v^2 + 80 v^3 + 385 v^4 (the
        positive-coefficient form of the kernel's potential about its edge), zero
        beyond n = 4. The Newtonian values are computed first and replaced lane
        by lane (a select, so the infinities at s = 0 never enter a product)."""
        K = self.K
        e = self.e
        e("T " + ", ".join(f"F{n}" for n in range(K + 1)) + ";")
        e("if constexpr (!K1) {")
        e("const T s_ = hot_fma(X, X, hot_fma(Y, Y, hot_fma(Z, Z, e2)));")
        e("const T u_ = hot_rsq(s_);")
        e("const T is_ = u_ * u_;")
        e("F0 = -u_;")
        if K >= 1:
            e("F1 = u_ * is_;")
        for n in range(1, K):
            e(f"F{n + 1} = (F{n} * is_) * {lit(-(2 * n + 1))};")
        e("} else {")
        e("const T s_ = hot_fma(X, X, hot_fma(Y, Y, Z * Z));")
        e("const T u_ = hot_rsq(s_);")
        e("const T is_ = u_ * u_;")
        e("F0 = -u_;")
        if K >= 1:
            e("F1 = u_ * is_;")
        for n in range(1, K):
            e(f"F{n + 1} = (F{n} * is_) * {lit(-(2 * n + 1))};")
        e("if (s_ < e2) {")
        e("const T ie_ = hot_rsq(e2);")
        e("const T ie2_ = ie_ * ie_;")
        e("const T v_ = (e2 - s_) * ie2_;")
        # Q^(n)(v) * 2^n / 256 with the sign of F_n, highest power first
        polys = [(-1, [1.0, 0.5, 0.375, 0.3125, 1.50390625]),
                 (1, [1.0, 1.5, 1.875, 12.03125]),
                 (-1, [3.0, 7.5, 72.1875]),
                 (1, [15.0, 288.75]),
                 (-1, [577.5])]
        e("T iep_ = ie_;")
        for n in range(0, K + 1):
            if n < len(polys):
                sg, c = polys[n]
                h = lit(c[-1])
                for co in reversed(c[:-1]):
                    h = f"hot_fma(v_, {h}, {lit(co)})"
                e(f"F{n} = {'-' if sg < 0 else ''}(iep_ * {h});")
                if n + 1 <= K and n + 1 < len(polys):
                    e("iep_ = iep_ * ie2_;")
            else:
                e(f"F{n} = T(0);")
        e("}")
        e("}")
        # powers of X
        if K >= 2:
            e("const T X2 = X * X;")
        for k in range(3, K + 1):
            e(f"const T X{k} = X{k - 1} * X;")

    def xpow(self, k):
        return "X" if k == 1 else f"X{k}"

    def derivs(self, consume):
        """Emit R_{t,u,v} for all t+u+v <= K, calling consume(t,u,v,name)."""
        K = self.K
        e = self.e
        # z chain rows are emitted lazily: row v needs rows v-1 and v-2
        def zname(v, n):
            return f"F{n}" if v == 0 else f"Z{v}_{n}"

        def yname(v, u, n):
            return zname(v, n) if u == 0 else f"Y{v}_{u}_{n}"

        for v in range(0, K + 1):
            if v >= 1 and self.row_barriers:
                e("HOT_ROW_BARRIER();")
            if v >= 1:
                for n in range(0, K - v + 1):
                    if v == 1:
                        e(f"const T Z1_{n} = Z * F{n + 1};")
                    else:
                        e(f"const T Z{v}_{n} = hot_fma(Z, {zname(v - 1, n + 1)}, {lit(v - 1)} * {zname(v - 2, n + 1)});")
            for u in range(0, K - v + 1):
                if u >= 1:
                    for n in range(0, K - v - u + 1):
                        if u == 1:
                            e(f"const T Y{v}_1_{n} = Y * {zname(v, n + 1)};")
                        else:
                            e(f"const T Y{v}_{u}_{n} = hot_fma(Y, {yname(v, u - 1, n + 1)}, {lit(u - 1)} * {yname(v, u - 2, n + 1)});")
                for t in range(0, K - v - u + 1):
                    name = f"R{t}_{u}_{v}"
                    terms = []
                    for j in range(0, t // 2 + 1):
                        c = math.factorial(t) // (math.factorial(j) * math.factorial(t - 2 * j)) / 2 ** j
                        terms.append((c, t - 2 * j, yname(v, u, t - j)))
                    # first term
                    c, px, yv = terms[0]
                    if px == 0:
                        expr = yv if c == 1 else f"{lit(c)} * {yv}"
                    else:
                        xp = self.xpow(px)
                        expr = f"{xp} * {yv}" if c == 1 else f"({lit(c)} * {xp}) * {yv}"
                    e(f"T {name} = {expr};")
                    for c, px, yv in terms[1:]:
                        if px == 0:
                            e(f"{name} = hot_fma({lit(c)}, {yv}, {name});")
                        else:
                            xp = self.xpow(px)
                            co = xp if c == 1 else f"({lit(c)} * {xp})"
                            e(f"{name} = hot_fma({co}, {yv}, {name});")
                    consume(t, u, v, name)


ROW_BARRIER_MIN_P = 7


def gen_fwd(P):
    K = P + 1
    em = Emitter(K, row_barriers=P >= ROW_BARRIER_MIN_P)
    em.radial()

    def consume(t, u, v, r):
        if t >= 1:
            em.e(f"ax = hot_fma(M[{slot(t - 1, u, v)}], {r}, ax);")
        if u >= 1:
            em.e(f"ay = hot_fma(M[{slot(t, u - 1, v)}], {r}, ay);")
        if v >= 1:
            em.e(f"az = hot_fma(M[{slot(t, u, v - 1)}], {r}, az);")
        if t + u + v <= P:
            em.e(f"if constexpr (POT) ph = hot_fma(M[{slot(t, u, v)}], {r}, ph);")

    em.derivs(consume)
    return em.lines


PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def gen_sink_adj(P):
    K = P + 2
    em = Emitter(K, row_barriers=P >= ROW_BARRIER_MIN_P)
    em.radial()
    for k, l in PAIRS:
        em.e(f"T H{k}{l} = T(0);")

    def consume(t, u, v, r):
        b = [t, u, v]
        for k, l in PAIRS:
            a = list(b)
            a[k] -= 1
            a[l] -= 1
            if min(a) < 0 or sum(a) > P:
                continue
            em.e(f"H{k}{l} = hot_fma(M[{slot(*a)}], {r}, H{k}{l});")

    em.derivs(consume)
    em.e("gx = hot_fma(H00, bx, hot_fma(H01, by, hot_fma(H02, bz, gx)));")
    em.e("gy = hot_fma(H01, bx, hot_fma(H11, by, hot_fma(H12, bz, gy)));")
    em.e("gz = hot_fma(H02, bx, hot_fma(H12, by, hot_fma(H22, bz, gz)));")
    return em.lines


def gen_cell_adj(P):
    K = P + 1
    em = Emitter(K)
    em.radial()
    remaining = {}
    for n in range(P + 1):
        for a in range(n, -1, -1):
            for b_ in range(n - a, -1, -1):
                remaining[slot(a, b_, n - a - b_)] = 3
    bname = ["bx", "by", "bz"]

    # each derivative goes straight into the row entries it feeds (per-sink
    # partial sums would stay live until their z term arrives with the next
    # z row)
    def consume(t, u, v, r):
        b = [t, u, v]
        for k in range(3):
            a = list(b)
            a[k] -= 1
            if a[k] < 0:
                continue
            s = slot(*a)
            em.e(f"row[{s}] = hot_fma({bname[k]}, {r}, row[{s}]);")
            remaining[s] -= 1

    em.derivs(consume)
    assert all(v == 0 for v in remaining.values())
    return em.lines


def gen_p2m_order(N):
    """acc[k] += m dx^a dy^b dz^c for the order-N slots, a descending, then b
    descending: the mass rides on the x powers (mx_a = m dx^a), and each slot
    takes one product with the y power and one fused multiply-add with the z
    power (two FP64 operations per slot)."""
    L = ["  const double mx0 = m;"]
    for k in range(1, N + 1):
        L.append(f"  const double mx{k} = mx{k - 1} * dx;")
    for name, var in (("py", "dy"), ("pz", "dz")):
        L.append(f"  const double {name}0 = 1.0;")
        for k in range(1, N + 1):
            L.append(f"  const double {name}{k} = {name}{k - 1} * {var};")
    k = 0
    for a in range(N, -1, -1):
        for b in range(N - a, -1, -1):
            c = N - a - b
            xy = f"mx{a}" if b == 0 else f"(mx{a} * py{b})"
            if c == 0:
                L.append(f"  acc[{k}] += {xy};")
            else:
                L.append(f"  acc[{k}] = fma({xy}, pz{c}, acc[{k}]);")
            k += 1
    return L


def gen_m2m_order(N):
    """Re-centre a child's moments (shift = child centre - parent centre) into
    the order-N slots: acc[alpha] += sum_{beta <= alpha} C(alpha,beta)
    shift^(alpha-beta) M[beta]. Source-major: each child moment M[beta] is
    read once and scattered into the slots alpha >= beta with one fused
    multiply-add each (the binomial weight folded into the shift monomial),
    which keeps few child moments live at a time."""
    L = []
    for name, var in (("px", "dx"), ("py", "dy"), ("pz", "dz")):
        L.append(f"  const double {name}0 = 1.0;")
        for k in range(1, N + 1):
            L.append(f"  const double {name}{k} = {name}{k - 1} * {var};")
    slots = []
    for a in range(N, -1, -1):
        for b in range(N - a, -1, -1):
            slots.append((a, b, N - a - b))
    for n2 in range(N + 1):
        for a2 in range(n2, -1, -1):
            for b2 in range(n2 - a2, -1, -1):
                c2 = n2 - a2 - b2
                L.append(f"  {{ const double m = M[{slot(a2, b2, c2)}];")
                for k, (a, b, c) in enumerate(slots):
                    if a < a2 or b < b2 or c < c2:
                        continue
                    co = math.comb(a, a2) * math.comb(b, b2) * math.comb(c, c2)
                    mono = f"((px{a - a2} * py{b - b2}) * pz{c - c2})"
                    w = mono if co == 1 else f"({float(co)!r} * {mono})"
                    L.append(f"    acc[{k}] = fma({w}, m, acc[{k}]);")
                L.append("  }")
    return L


def gen_m2mT_order(P, N):
    """Transpose of the re-centring for the order-N output slots beta:
    acc[beta] += sum_{alpha >= beta, |alpha| <= P} C(alpha,beta)
    shift^(alpha-beta) Mbar[alpha]  (shift = child centre - parent centre).
    Source-major like the re-centring itself: each parent cotangent
    Mbar[alpha] is read once and scattered into the slots beta <= alpha with
    one fused multiply-add each."""
    L = []
    for name, var in (("px", "dx"), ("py", "dy"), ("pz", "dz")):
        L.append(f"  const double {name}0 = 1.0;")
        for k in range(1, P - N + 1):
            L.append(f"  const double {name}{k} = {name}{k - 1} * {var};")
    outs = []
    for b0 in range(N, -1, -1):
        for b1 in range(N - b0, -1, -1):
            outs.append((b0, b1, N - b0 - b1))
    for n in range(N, P + 1):
        for a0 in range(n, -1, -1):
            for a1 in range(n - a0, -1, -1):
                a2 = n - a0 - a1
                L.append(f"  {{ const double mb = Mb[{slot(a0, a1, a2)}];")
                for k, (b0, b1, b2) in enumerate(outs):
                    if a0 < b0 or a1 < b1 or a2 < b2:
                        continue
                    co = math.comb(a0, b0) * math.comb(a1, b1) * math.comb(a2, b2)
                    mono = f"((px{a0 - b0} * py{a1 - b1}) * pz{a2 - b2})"
                    w = mono if co == 1 else f"({float(co)!r} * {mono})"
                    L.append(f"    acc[{k}] = fma({w}, mb, acc[{k}]);")
                L.append("  }")
    return L


def gen_p2mT(P):
    """Moment cotangents to one particle at offset d from the cell centre:
    g_k += sum_alpha Mb[alpha] alpha_k d^(alpha-e_k), gm += sum_alpha Mb[alpha] d^alpha."""
    L = []
    for name, var in (("px", "dx"), ("py", "dy"), ("pz", "dz")):
        L.append(f"  const double {name}0 = 1.0;")
        for k in range(1, P + 1):
            L.append(f"  const double {name}{k} = {name}{k - 1} * {var};")
    for n in range(P + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                c = n - a - b
                s_ = slot(a, b, c)
                L.append(f"  gm = fma(Mb[{s_}], (px{a} * py{b}) * pz{c}, gm);")
                if a:
                    L.append(f"  gx = fma({float(a)!r} * Mb[{s_}], (px{a - 1} * py{b}) * pz{c}, gx);")
                if b:
                    L.append(f"  gy = fma({float(b)!r} * Mb[{s_}], (px{a} * py{b - 1}) * pz{c}, gy);")
                if c:
                    L.append(f"  gz = fma({float(c)!r} * Mb[{s_}], (px{a} * py{b}) * pz{c - 1}, gz);")
    return L


def _count_ops(lines):
    """FP operations in emitted lines: fused multiply-add = 2, multiply or
    add = 1, reciprocal square root = 1; multiplications or FMAs by the
    literal 1 are not counted as multiplies."""
    n = 0
    for l in lines:
        n += 2 * l.count("hot_fma(") - l.count("hot_fma(T(1.0),")
        n += l.count(" * ") - l.count("T(1.0) * ")
        n += l.count("hot_rsq(")
    return n



def _plummer_only(lines):
    """The emitted lines without the K1 branch of the radial functions."""
    out, skip, depth = [], False, 0
    for l in lines:
        t = l.strip()
        if not skip and t == "} else {":
            skip, depth = True, 1
            continue
        if skip:
            depth += t.count("{") - t.count("}")
            if depth <= 0:
                skip = False
            continue
        out.append(l)
    return out


def flops_m2p(P):
    """FP32 operations per (sink, cell) of the forward expansion kernel without
    the potential, Plummer softening: the generated expansion plus the
    per-interaction setup of the kernel (scaled R: 3 multiplies and 3 adds;
    result scaling: 3 multiplies; compensated accumulation: 4 adds for each of
    3 components)."""
    body = [l for l in _plummer_only(gen_fwd(P)) if "if constexpr (POT)" not in l]
    return _count_ops(body) + 6 + 3 + 12


def flops_p2p():
    """FP32 operations per (sink, source) pair of the pair kernel without the
    potential: r = s + t (3 adds), r^2 + eps^2 (3 FMAs), rsq, m*inv, inv*inv,
    times (3 multiplies), accumulation (3 FMAs)."""
    return 3 + 6 + 1 + 3 + 6


def main(out_path):
    parts = ["// Generated by gen_expansions.py -- do not edit.",
             "#pragma once",
             "#ifndef HOT_ROW_BARRIER",
             "#define HOT_ROW_BARRIER() __builtin_amdgcn_sched_barrier(0)",
             "#endif",
             "namespace hot {",
             ""]
    parts.append("template <int P, typename T, bool POT, bool K1 = false>")
    parts.append("__device__ __forceinline__ void expansion_fwd(T X, T Y, T Z, T e2, "
                 "const T* __restrict__ M, T& ax, T& ay, T& az, T& ph) {")
    for P in range(PMAX + 1):
        kw = "if constexpr" if P == 0 else "} else if constexpr"
        parts.append(f"  {kw} (P == {P}) {{")
        parts += ["  " + l for l in gen_fwd(P)]
    parts.append("  }")
    parts.append("}")
    parts.append("")
    parts.append("template <int P, typename T, bool K1 = false>")
    parts.append("__device__ __forceinline__ void expansion_sink_adj(T X, T Y, T Z, T e2, "
                 "const T* __restrict__ M, T bx, T by, T bz, T& gx, T& gy, T& gz) {")
    for P in range(PMAX + 1):
        kw = "if constexpr" if P == 0 else "} else if constexpr"
        parts.append(f"  {kw} (P == {P}) {{")
        parts += ["  " + l for l in gen_sink_adj(P)]
    parts.append("  }")
    parts.append("}")
    parts.append("")
    parts.append("template <int P, typename T, bool K1 = false>")
    parts.append("__device__ __forceinline__ void expansion_cell_adj(T X, T Y, T Z, T e2, "
                 "T bx, T by, T bz, T* row) {")
    for P in range(PMAX + 1):
        kw = "if constexpr" if P == 0 else "} else if constexpr"
        parts.append(f"  {kw} (P == {P}) {{")
        parts += ["  " + l for l in gen_cell_adj(P)]
    parts.append("  }")
    parts.append("}")
    parts.append("")
    for N in range(PMAX + 1):
        parts.append(f"__device__ __forceinline__ void p2m_order{N}(double dx, double dy, double dz, "
                     "double m, double* acc) {")
        parts += gen_p2m_order(N)
        parts.append("}")
        parts.append(f"__device__ __forceinline__ void m2m_order{N}(const double* __restrict__ M, "
                     "double dx, double dy, double dz, double* acc) {")
        parts += gen_m2m_order(N)
        parts.append("}")
    for P in range(PMAX + 1):
        for N in range(P + 1):
            parts.append(f"__device__ __forceinline__ void m2mT_p{P}_order{N}(const double* __restrict__ Mb, "
                         "double dx, double dy, double dz, double* acc) {")
            parts += gen_m2mT_order(P, N)
            parts.append("}")
        parts.append(f"__device__ __forceinline__ void p2mT_p{P}(const double* __restrict__ Mb, "
                     "double dx, double dy, double dz, double& gx, double& gy, double& gz, double& gm) {")
        parts += gen_p2mT(P)
        parts.append("}")
    parts.append("")
    parts.append("}  // namespace hot")
    text = "\n".join(parts) + "\n"
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    tmp = out_path + ".tmp"
    with open(tmp, "w") as f:
        f.write(text)
    os.replace(tmp, out_path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "generated", "expansions.h"))
