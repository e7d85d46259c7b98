"""Writes sym_rules.hpp: the fully symmetric quadrature rules of the convection kernels.

Volume rules.  The volume integrand of the operator, (u (x) w) : grad(phi) for w, u and phi of
degree k, is a polynomial of degree 3k-1, so any rule exact to that degree gives the same
operator up to rounding.  The collapsed Gauss-Jacobi product rule needs ceil(3k/2)^d points;
the fully symmetric rules below (invariant under every permutation of the simplex vertices,
positive weights, every point inside the simplex) need fewer:

    2D  k = 1: 3 (collapsed 4)    k = 2: 7 (9)     k = 3: 16 (25)    k = 4: 28 (36)
        k = 5: 42 (64)
    3D  k = 1: 4 (8)              k = 2: 14 (27)   k = 3: 46 (125)

Facet rules (3D).  The upwind value is taken pointwise, so the facet rule is part of the
operator's definition; on a triangular facet it is the symmetric rule of degree 3k where one
needs fewer points than the collapsed rule with ceil((3k+1)/2)^2: k = 2 the 12-point degree-6
rule, k = 3 the 19-point degree-9 rule of D. A. Dunavant (Int. J. Numer. Methods Eng. 21,
1985), weights summing to 1.

A rule is given by its orbits under the vertex permutations, each a barycentric generator
with free parameters ('3' the centroid, '21' (a, a, 1-2a), '111' (a, b, 1-a-b); '4' the
centroid, '31' (a, a, a, 1-3a), '22' (a, a, 1/2-a, 1/2-a), '211' (a, a, b, 1-2a-b)), and by
starting values of those parameters that a random-start least-squares search found (positions
by Levenberg-Marquardt, weights by linear least squares at each step).  This script refines
parameters and weights by Gauss-Newton steps in 60-digit arithmetic against the exact moments
of the monomials on the reference simplex,

    int x^i y^j = i! j! / (i+j+2)!,    int x^i y^j z^l = i! j! l! / (i+j+l+3)!,

checks exactness to 1e-40, positive weights and interior points, and writes the expanded
points (reference coordinates = barycentric coordinates 1..d) and weights as long double
literals.

    python gen_sym_rules.py > sym_rules.hpp
"""
import itertools
import sys

import mpmath as mp

mp.mp.dps = 60

# (dim, k): list of (orbit type, starting parameters); weights are solved for
RULES = {
    (2, 1): [("21", [0.16666666666666666])],
    (2, 2): [("3", []), ("21", [0.10128650732345626]), ("21", [0.47014206410511444])],
    (2, 3): [("3", []), ("21", [0.4592925882927678]), ("21", [0.1705693077518829]),
             ("21", [0.05054722831706721]), ("111", [0.008394777410064983, 0.7284923929554489])],
    (2, 4): [("3", []), ("21", [0.211202368345754]), ("21", [0.10523213974936128]),
             ("21", [0.029132577733838472]), ("21", [0.4964082121896513]),
             ("21", [0.43821104894017354]), ("111", [0.009252951305720096, 0.1518192044856569]),
             ("111", [0.0463970358405466, 0.29407958108856036])],
    (2, 5): [("21", [0.06179988309089579]), ("21", [0.4176447193403893]),
             ("21", [0.2734775283089308]), ("21", [0.019390961248661156]),
             ("21", [0.17720553241294396]), ("21", [0.4889639103622024]),
             ("111", [0.09291624935686842, 0.3368614597964482]),
             ("111", [0.17226668782115825, 0.7706085547747088]),
             ("111", [0.11897449769695961, 0.8797571713697192]),
             ("111", [0.014646950055685488, 0.6869801678083242])],
    (3, 1): [("31", [0.1381966011250105])],
    (3, 2): [("31", [0.3108859192633004]), ("31", [0.0927352503108908]),
             ("22", [0.04550370412565067])],
    (3, 3): [("31", [0.18368219959177393]), ("31", [0.0890842680038524]),
             ("31", [0.3150760322173066]), ("31", [0.030376367946228715]),
             ("22", [0.43884998942322245]), ("211", [0.022674246187050374, 0.22923965490894646]),
             ("211", [0.20580974356370157, 0.0162315274171111])],
}

# 3D facet rules, k: orbits on the triangle (degree 3k)
FACET_RULES = {
    2: [("21", [0.06308901449150214]), ("21", [0.24928674517090987]),
        ("111", [0.053145049844816925, 0.3103524510337838])],
    3: [("3", []), ("21", [0.04472951339445053]), ("21", [0.18820353561903191]),
        ("21", [0.43708959149293103]), ("21", [0.4896825191987205]),
        ("111", [0.036838412054736404, 0.221962989160761])],
}


def generators(dim, kind, p):
    one = mp.mpf(1)
    if dim == 2:
        if kind == "3":
            return (one / 3,) * 3
        if kind == "21":
            return (p[0], p[0], one - 2 * p[0])
        if kind == "111":
            return (p[0], p[1], one - p[0] - p[1])
    else:
        if kind == "4":
            return (one / 4,) * 4
        if kind == "31":
            return (p[0],) * 3 + (one - 3 * p[0],)
        if kind == "22":
            return (p[0], p[0], one / 2 - p[0], one / 2 - p[0])
        if kind == "211":
            return (p[0], p[0], p[1], one - 2 * p[0] - p[1])
    raise ValueError(kind)


NPAR = {"3": 0, "21": 1, "111": 2, "4": 0, "31": 1, "22": 1, "211": 2}


def orbit_points(dim, kind, p):
    """Distinct permutations of the generator, in lexicographic order of the permutation."""
    g = generators(dim, kind, p)
    seen, out = set(), []
    for perm in itertools.permutations(range(dim + 1)):
        b = tuple(g[i] for i in perm)
        key = tuple(mp.nstr(v, 40) for v in b)
        if key not in seen:
            seen.add(key)
            out.append(b)
    return out


def monomials(dim, deg):
    if dim == 2:
        return [(i, s - i) for s in range(deg + 1) for i in range(s + 1)]
    return [(i, j, s - i - j) for s in range(deg + 1) for i in range(s + 1)
            for j in range(s + 1 - i)]


def exact_moment(e):
    num = 1
    for a in e:
        num *= mp.factorial(a)
    return num / mp.factorial(sum(e) + len(e))


def unpack(dim, spec, x):
    """x = all free positions, then one weight per orbit."""
    k, orbits = 0, []
    for kind, _ in spec:
        n = NPAR[kind]
        orbits.append((kind, x[k:k + n]))
        k += n
    return orbits, x[k:]


def residual(dim, spec, x, mons, exact):
    orbits, w = unpack(dim, spec, x)
    r = [-v for v in exact]
    for (kind, p), wo in zip(orbits, w):
        for b in orbit_points(dim, kind, p):
            xs = b[1:]
            for i, e in enumerate(mons):
                t = wo
                for a in range(dim):
                    if e[a]:
                        t *= xs[a] ** e[a]
                r[i] += t
    return r


def refine(dim, deg, spec, n_collapsed):
    mons = monomials(dim, deg)
    exact = [exact_moment(e) for e in mons]
    x = [mp.mpf(v) for _, p in spec for v in p]
    # starting weights: linear least squares at the starting positions
    npos = len(x)
    orbits, _ = unpack(dim, spec, x + [mp.mpf(0)] * len(spec))
    A = mp.matrix(len(mons), len(spec))
    for c, (kind, p) in enumerate(orbits):
        for b in orbit_points(dim, kind, p):
            for i, e in enumerate(mons):
                t = mp.mpf(1)
                for a in range(dim):
                    t *= b[1 + a] ** e[a]
                A[i, c] += t
    w = mp.lu_solve(A.T * A, A.T * mp.matrix(exact))
    x = x + [w[i] for i in range(len(spec))]
    h = mp.mpf(10) ** -28
    for it in range(40):
        r = residual(dim, spec, x, mons, exact)
        err = max(abs(v) for v in r)
        if err < mp.mpf(10) ** -50:
            break
        J = mp.matrix(len(mons), len(x))
        for c in range(len(x)):
            xp = list(x)
            xp[c] += h
            rp = residual(dim, spec, xp, mons, exact)
            for i in range(len(mons)):
                J[i, c] = (rp[i] - r[i]) / h
        dx = mp.lu_solve(J.T * J, -(J.T * mp.matrix(r)))
        x = [x[c] + dx[c] for c in range(len(x))]
    r = residual(dim, spec, x, mons, exact)
    err = max(abs(v) for v in r)
    orbits, w = unpack(dim, spec, x)
    pts, wts = [], []
    for (kind, p), wo in zip(orbits, w):
        for b in orbit_points(dim, kind, p):
            pts.append(b[1:])
            wts.append(wo)
    assert err < mp.mpf(10) ** -40, (dim, deg, err)
    assert all(v > 0 for v in wts), (dim, deg)
    assert all(min(b) > 0 and 1 - sum(b) > 0 for b in pts), (dim, deg)
    assert len(wts) < n_collapsed, (dim, deg)
    return pts, wts, err, npos


def write_rule(out, name, title, pts, wts):
    out.write("// %s\n" % title)
    out.write("inline constexpr long double %s_pts[] = {\n" % name)
    for b in pts:
        out.write("    " + ", ".join(mp.nstr(v, 24, strip_zeros=False) + "L" for v in b) + ",\n")
    out.write("};\ninline constexpr long double %s_wts[] = {\n" % name)
    for v in wts:
        out.write("    " + mp.nstr(v, 24, strip_zeros=False) + "L,\n")
    out.write("};\n\n")


def main():
    out = sys.stdout
    out.write("// Generated by gen_sym_rules.py (fully symmetric quadrature rules with positive\n"
              "// weights and interior points); do not edit.\n"
              "#pragma once\n\nnamespace dgref {\n\n")
    vol, fac = [], []
    for (dim, k), spec in sorted(RULES.items()):
        pts, wts, err, _ = refine(dim, 3 * k - 1, spec, max(1, (3 * k + 1) // 2) ** dim)
        name = "kVolRule%dd_k%d" % (dim, k)
        write_rule(out, name, "volume %dD, k = %d: degree %d, %d points (%s); max moment error %s"
                   % (dim, k, 3 * k - 1, len(wts), " + ".join(t[0] for t in spec), mp.nstr(err, 3)),
                   pts, wts)
        vol.append((dim, k, len(wts), name))
    for k, spec in sorted(FACET_RULES.items()):
        pts, wts, err, _ = refine(2, 3 * k, spec, max(1, (3 * k + 2) // 2) ** 2)
        name = "kFacRule3d_k%d" % k
        write_rule(out, name, "3D facet, k = %d: degree %d, %d points (%s), weights summing to 1; "
                   "max moment error %s" % (k, 3 * k, len(wts), " + ".join(t[0] for t in spec),
                                            mp.nstr(err, 3)), pts, [2 * v for v in wts])
        fac.append((k, len(wts), name))
    out.write("// points of the symmetric volume rule for (dim, k), 0 where there is none\n"
              "constexpr int sym_vol_points(int dim, int k) {\n")
    for dim, k, n, _ in vol:
        out.write("  if (dim == %d && k == %d) return %d;\n" % (dim, k, n))
    out.write("  return 0;\n}\n\n")
    out.write("// the symmetric volume rule for (dim, k): points [n][dim], weights [n]; false if none\n"
              "inline bool sym_vol_rule(int dim, int k, const long double** pts,\n"
              "                         const long double** wts) {\n")
    for dim, k, _, name in vol:
        out.write("  if (dim == %d && k == %d) { *pts = %s_pts; *wts = %s_wts; return true; }\n"
                  % (dim, k, name, name))
    out.write("  return false;\n}\n\n")
    out.write("// points of the symmetric 3D facet rule for k, 0 where there is none\n"
              "constexpr int sym_facet_points(int k) {\n")
    for k, n, _ in fac:
        out.write("  if (k == %d) return %d;\n" % (k, n))
    out.write("  return 0;\n}\n\n")
    out.write("// the symmetric 3D facet rule for k: points (s, t) [n][2], weights [n] summing to 1;\n"
              "// false if none\n"
              "inline bool sym_facet_rule(int k, const long double** pts, const long double** wts) {\n")
    for k, _, name in fac:
        out.write("  if (k == %d) { *pts = %s_pts; *wts = %s_wts; return true; }\n" % (k, name, name))
    out.write("  return false;\n}\n\n}  // namespace dgref\n")


if __name__ == "__main__":
    main()
