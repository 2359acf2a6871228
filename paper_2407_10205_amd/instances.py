"""Seeded synthetic Ising instances.

This module only draws inputs (couplings J, local fields h) with the
coefficient distributions of the problem families the paper benchmarks
(Table 2); it holds none of the annealer's arithmetic.  Every generator uses
``numpy.random.Generator(numpy.random.Philox(seed))`` so that the same seed
gives the same instance on every machine.

Conventions: J is a dense symmetric float64 [N, N] array with a zero
diagonal, h a float64 [N] array; the Ising energy is
E(s) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i (Eq. 2).
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.Philox(int(seed)))


def _sym(U):
    """Mirror the strict upper triangle of U into a symmetric matrix."""
    T = np.triu(U, 1)
    return T + T.T


def sk_pm1(N, seed):
    """Sherrington-Kirkpatrick spin glass, J_ij uniform in {-1, +1}, h = 0
    (the sk_ising family of Table 2)."""
    g = rng(seed)
    U = g.integers(0, 2, size=(N, N)).astype(np.float64) * 2.0 - 1.0
    return _sym(U), np.zeros(N)


def er_maxcut(N, p, seed, signed=False):
    """Max-cut on an Erdos-Renyi graph G(N, p) as an Ising problem.

    Edge weights w_ij = +1 (or uniform +-1 when signed); maximising the cut
    sum_{i<j} w_ij (1 - s_i s_j)/2 is minimising E with J_ij = -w_ij, h = 0,
    and cut = (W - E)/2 with W = sum of the weights (maxcut_dense family).
    """
    g = rng(seed)
    A = (g.random((N, N)) < p).astype(np.float64)
    if signed:
        A *= g.integers(0, 2, size=(N, N)) * 2.0 - 1.0
    W = _sym(A)
    return -W, np.zeros(N)


def sk_gauss_fixed(N, seed, frac_bits=5, bits=8):
    """SK with Gaussian couplings quantised to a signed fixed-point grid.

    J_int = clamp(rint(2^f z), -(2^(bits-1)), 2^(bits-1)-1) with z ~ N(0, 1)
    and J = J_int 2^-f; h_int uniform on [-2^f, 2^f] so h lies in [-1, 1]
    on the same grid (the spin_model family with fractional coefficients).
    """
    g = rng(seed)
    sc = float(2 ** frac_bits)
    lo, hi = -(2 ** (bits - 1)), 2 ** (bits - 1) - 1
    Z = g.standard_normal((N, N))
    Ji = np.clip(np.rint(Z * sc), lo, hi)
    hi_ = g.integers(-int(sc), int(sc) + 1, size=N).astype(np.float64)
    return _sym(Ji) / sc, hi_ / sc


def regular3_pm1(N, seed, with_field=True):
    """Random 3-regular graph (pairing model with restarts), J = +-1 on its
    edges, h uniform in {-1, 0, 1} (the maxcut_d3 family with signs).
    N must be even."""
    if N % 2:
        raise ValueError("a 3-regular graph needs an even number of vertices")
    g = rng(seed)
    while True:
        stubs = np.repeat(np.arange(N), 3)
        g.shuffle(stubs)
        a, b = stubs[0::2], stubs[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        if len(set(zip(lo.tolist(), hi.tolist()))) != len(lo):
            continue
        break
    J = np.zeros((N, N))
    sgn = g.integers(0, 2, size=lo.shape[0]) * 2.0 - 1.0
    J[lo, hi] = sgn
    J[hi, lo] = sgn
    h = g.integers(-1, 2, size=N).astype(np.float64) if with_field else np.zeros(N)
    return J, h


def uniform_fixed(N, seed, frac_bits=8, with_field=True):
    """Couplings and fields uniform on [-1, 1] rounded to the 2^-f grid
    (the spin_model family of Table 2)."""
    g = rng(seed)
    sc = float(2 ** frac_bits)
    U = np.rint(g.uniform(-1.0, 1.0, size=(N, N)) * sc) / sc
    h = np.rint(g.uniform(-1.0, 1.0, size=N) * sc) / sc if with_field else np.zeros(N)
    return _sym(U), h


def regular3_graph(N, seed):
    """Adjacency matrix of a random 3-regular graph (pairing model with
    restarts; N even)."""
    J, _ = regular3_pm1(N, seed, with_field=False)
    return np.abs(J)


def nae_3_sat(N, seed, alpha=2.0, planted=True):
    """NAE-3-SAT as an Ising instance (clause-to-triangle reduction).

    Clause k holds three distinct variables v with literal signs t (literal
    value t s_v).  It is not-all-equal satisfied iff its literals are not
    all equal; the sum of its three pairwise literal products is then -1,
    else +3.  With J_ij = -(sum of t_i t_j over the clauses that contain the
    pair i, j) and h = 0, Eq. 2 gives E(s) = sum over clauses of that pair
    sum, so E >= -M for M clauses, with equality exactly when every clause
    is NAE-satisfied.  Couplings are small integers (pairs shared by several
    clauses add up), the coefficient set of the family in Table 2.

    M = round(alpha N) clauses on uniformly drawn variable triples with fair
    literal signs; planted=True keeps a clause only if a hidden uniform
    assignment z NAE-satisfies it, so E(z) = -M is the ground energy.
    Returns (J, h, M, z, clauses) with clauses an [M][3][2] array of
    (variable, sign).
    """
    if N < 3:
        raise ValueError("NAE-3-SAT needs at least three variables")
    g = rng(seed)
    z = g.choice([-1, 1], size=N)
    M = max(1, int(round(alpha * N)))
    clauses = []
    while len(clauses) < M:
        v = g.choice(N, size=3, replace=False)
        t = g.choice([-1, 1], size=3)
        lit = t * z[v]
        if planted and lit[0] == lit[1] == lit[2]:
            continue
        clauses.append(np.stack([v, t], axis=1))
    C = np.array(clauses, dtype=np.int64)
    J = np.zeros((N, N))
    for cl in C:
        for a in range(3):
            for b in range(a + 1, 3):
                i, j = cl[a, 0], cl[b, 0]
                w = float(cl[a, 1] * cl[b, 1])
                J[i, j] -= w
                J[j, i] -= w
    return J, np.zeros(N), M, z.astype(np.float64), C


# Table 2 families.  The table lists the problem's coefficients; as for the
# max-cut rows (graph weights w, Ising couplings J = -w), every family enters
# Eq. 2 with couplings -w, so that all of them are frustrated.
def table2_family(name, N, seed, frac_bits=6):
    """Instance of a Table 2 family of size N: (J, h) on the 2^-frac_bits
    grid (fractional families are rounded onto it)."""
    g = rng(seed)
    if name == "maxcut_dense":          # unweighted max-cut on G(N, 1/2)
        return er_maxcut(N, 0.5, seed)
    if name == "maxcut_d3":             # unweighted max-cut on a cubic graph
        return -regular3_graph(N, seed), np.zeros(N)
    if name == "sk_bool":               # w_ij in {0, 1}, iid fair coin
        W = g.integers(0, 2, size=(N, N)).astype(np.float64)
        return -_sym(W), np.zeros(N)
    if name == "sk_ising":              # w_ij in {-1, +1}
        return sk_pm1(N, seed)
    if name == "sk_uniform":            # w_ij = 0 or U(0, 1), each with probability 1/2
        sc = float(2 ** frac_bits)
        W = np.where(g.random((N, N)) < 0.5, 0.0, np.rint(g.random((N, N)) * sc) / sc)
        return -_sym(W), np.zeros(N)
    if name == "spin_model":            # w_ij, h_i uniform on [-1, 1]
        J, h = uniform_fixed(N, seed, frac_bits=frac_bits)
        return -J, h
    if name == "nae_3_sat":             # planted NAE-3-SAT, 2 N clauses (reduction above: already E = pair sums)
        J, h, _, _, _ = nae_3_sat(N, seed)
        return J, h
    raise ValueError(f"unknown family {name}")


TABLE2_FAMILIES = ("maxcut_dense", "maxcut_d3", "sk_bool", "sk_ising", "sk_uniform", "nae_3_sat", "spin_model")


def random_field_pm1(N, seed):
    """Integer fields in {-1, 0, 1} drawn independently (used to add h to an
    integer coupling family)."""
    return rng(seed).integers(-1, 2, size=N).astype(np.float64)


def planted_loops(N, seed, alpha=0.4, dense=False, min_len=4):
    """Planted-solution instance from frustrated loops (Hen et al., PRA 92,
    042325, 2015), in the convention E = -sum_{i<j} J_ij s_i s_j.

    Loops are cycles cut out of random walks (no immediate backtracking) on a
    base graph -- a random 3-regular graph (sparse) or the complete graph
    (dense).  Each loop adds +1 to the couplings of its edges except one
    random edge, which gets -1: with all spins +1 the loop satisfies every
    bond but one, which is the best any configuration can do on a frustrated
    cycle, so the sum over loops is minimised by s = +1 with energy
    -sum_loops (len - 2).  A random gauge t (J_ij -> t_i t_j J_ij) hides the
    solution: the planted state is t with the same energy.

    Returns (J, h, E_planted, t) with h = 0 and integer couplings.
    """
    g = rng(seed)
    if dense:
        def step(u, prev):
            while True:
                w = int(g.integers(0, N))
                if w != u and w != prev:
                    return w
    else:
        M = N + (N % 2)
        base, _ = regular3_pm1(M, int(g.integers(0, 2**31)), with_field=False)
        nbrs = [np.nonzero(base[i])[0][np.nonzero(base[i])[0] < N] for i in range(N)]

        def step(u, prev):
            cand = [int(w) for w in nbrs[u] if w != prev]
            if not cand:
                cand = [int(w) for w in nbrs[u]]
            return cand[int(g.integers(0, len(cand)))]
    J = np.zeros((N, N))
    E = 0
    loops = 0
    target = max(1, int(round(alpha * N)))
    tries = 0
    while loops < target and tries < 100 * target:
        tries += 1
        start = int(g.integers(0, N))
        path, pos, prev = [start], {start: 0}, -1
        u = start
        for _ in range(4 * N):
            w = step(u, prev)
            if w in pos:
                cyc = path[pos[w]:]
                break
            pos[w] = len(path)
            path.append(w)
            prev, u = u, w
        else:
            continue
        if len(cyc) < min_len:
            continue
        edges = [(cyc[i], cyc[(i + 1) % len(cyc)]) for i in range(len(cyc))]
        bad = int(g.integers(0, len(edges)))
        for e_i, (a, b) in enumerate(edges):
            v = -1.0 if e_i == bad else 1.0
            J[a, b] += v
            J[b, a] += v
        E -= len(cyc) - 2
        loops += 1
    t = g.integers(0, 2, size=N) * 2.0 - 1.0
    J = J * np.outer(t, t)
    return J, np.zeros(N), int(E), t.astype(np.int8)
