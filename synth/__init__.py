"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays out model parameters.  It
holds none of the method's arithmetic: no Pauli algebra, no Jordan-Wigner
mapping, no sector indexing and no operator application.  Both the oracle
and the GPU path read their inputs from here, so a parity test compares two
independent computations on identical bytes.

Conventions (spin-orbital layout used by the molecular Hamiltonian of
Eq. second_quantized_hamiltonian in the paper's Section 2.1):

* spatial orbital p with spin alpha is spin-orbital p, with spin beta it is
  spin-orbital n_orb + p ("blocked" order, so that the alpha string is the
  low half of a basis index and the beta string the high half, matching the
  spin-resolved product basis of Section 2.4);
* spatial two-electron integrals are in chemists' notation g[p,q,r,s] =
  (pq|rs) with the 8-fold permutational symmetry of real orbitals;
* the spin-orbital tensor h2[P,Q,R,S] is the coefficient of
  1/2 a+_P a+_Q a_R a_S, i.e. (p_P p_S | p_Q p_R) when spin(P) = spin(S)
  and spin(Q) = spin(R), and 0 otherwise.
"""

import numpy as np

__all__ = [
    "molecular_integrals",
    "spin_orbital_integrals",
    "molecular_spin_integrals",
    "hubbard_spatial_integrals",
    "hubbard_spin_integrals",
    "tfim_terms",
    "random_state",
    "random_pauli_strings",
    "neel_occupations",
    "pes_integrals",
    "excitation_generators",
    "excitation_masks",
    "mlp_init",
]


def _orbit_representatives(n_orb):
    """Index arrays (a, b, c, d) such that g[a, b, c, d] is the canonical
    representative of the 8-fold permutation orbit of each (p, q, r, s):
    ordered pairs, then the ordered pair of pairs."""
    p, q, r, s = np.indices((n_orb,) * 4)
    pq_hi, pq_lo = np.maximum(p, q), np.minimum(p, q)
    rs_hi, rs_lo = np.maximum(r, s), np.minimum(r, s)
    first_is_big = pq_hi * n_orb + pq_lo >= rs_hi * n_orb + rs_lo
    return (np.where(first_is_big, pq_hi, rs_hi), np.where(first_is_big, pq_lo, rs_lo),
            np.where(first_is_big, rs_hi, pq_hi), np.where(first_is_big, rs_lo, pq_lo))


def molecular_integrals(n_orb, seed, h_scale=1.0, g_scale=0.1):
    """Random real spatial integrals (h, g).

    h: symmetric, h[p,q] = h[q,p] ~ N(0, h_scale^2) drawn for p <= q.
    g: one N(0, g_scale^2) draw per 8-fold orbit, copied to all 8 index
       permutations (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq) = ...
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n_orb, n_orb)) * h_scale
    h = np.triu(a) + np.triu(a, 1).T
    raw = rng.standard_normal((n_orb,) * 4) * g_scale
    g = raw[_orbit_representatives(n_orb)]
    return h, g


def spin_orbital_integrals(h, g):
    """Spatial (h, g) -> spin-orbital (h1, h2) in the blocked layout."""
    n = h.shape[0]
    ns = 2 * n
    sp = np.arange(ns) % n          # spatial index of each spin-orbital
    spin = np.arange(ns) // n       # 0 = alpha, 1 = beta
    h1 = h[sp[:, None], sp[None, :]] * (spin[:, None] == spin[None, :])
    P, Q, R, S = np.indices((ns,) * 4)
    allowed = (spin[P] == spin[S]) & (spin[Q] == spin[R])
    h2 = np.where(allowed, g[sp[P], sp[S], sp[Q], sp[R]], 0.0)
    return np.ascontiguousarray(h1, dtype=np.float64), np.ascontiguousarray(h2, dtype=np.float64)


def molecular_spin_integrals(n_orb, seed):
    """Spin-orbital integrals of the synthetic molecular Hamiltonian."""
    h, g = molecular_integrals(n_orb, seed)
    return spin_orbital_integrals(h, g)


def _lattice_bonds(rows, cols, periodic):
    bonds = set()
    for r in range(rows):
        for c in range(cols):
            i = r * cols + c
            for dr, dc in ((0, 1), (1, 0)):
                rr, cc = r + dr, c + dc
                if periodic:
                    rr %= rows
                    cc %= cols
                elif rr >= rows or cc >= cols:
                    continue
                j = rr * cols + cc
                if i != j:
                    bonds.add((min(i, j), max(i, j)))
    return sorted(bonds)


def hubbard_spatial_integrals(rows, cols, t=1.0, u=4.0, periodic=True):
    """Fermi-Hubbard model as spatial integrals (sites row-major).

    H = -t sum_<ij>,sigma (a+_i a_j + h.c.) + U sum_i n_i,up n_i,down, so
    h[i,j] = -t on each bond (a bond counted once even if periodic wrapping
    reaches the same neighbour twice) and (ii|ii) = U.
    """
    n = rows * cols
    h = np.zeros((n, n))
    for i, j in _lattice_bonds(rows, cols, periodic):
        h[i, j] = h[j, i] = -t
    g = np.zeros((n,) * 4)
    for i in range(n):
        g[i, i, i, i] = u
    return h, g


def hubbard_spin_integrals(rows, cols, t=1.0, u=4.0, periodic=True):
    h, g = hubbard_spatial_integrals(rows, cols, t, u, periodic)
    h1, h2 = spin_orbital_integrals(h, g)
    # With only on-site (ii|ii) integrals the same-spin entries h2[P,P,P,P]
    # multiply a+_P a+_P = 0; they are harmless but kept for fidelity.
    return h1, h2


def tfim_terms(n_sites, j=0.25, h=1.0):
    """Open-chain transverse-field Ising model J sum Z_i Z_i+1 + h sum X_i.

    Returned as letter strings (one char per qubit, qubit 0 first) with real
    coefficients; this is input data, not algebra.
    """
    terms = []
    for i in range(n_sites - 1):
        s = ["I"] * n_sites
        s[i] = s[i + 1] = "Z"
        terms.append(("".join(s), complex(j)))
    for i in range(n_sites):
        s = ["I"] * n_sites
        s[i] = "X"
        terms.append(("".join(s), complex(h)))
    return terms


def random_state(dim, seed):
    """(N(0,1) + i N(0,1)) per amplitude, normalised in float64."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    v /= np.sqrt(np.vdot(v, v).real)
    return v.astype(np.complex128)


def random_pauli_strings(n_strings, n_qubits, seed, with_phase=True):
    """Random letter strings as uint8 arrays (0=I, 1=X, 2=Y, 3=Z) and Z4 phases."""
    rng = np.random.default_rng(seed)
    letters = rng.integers(0, 4, size=(n_strings, n_qubits), dtype=np.uint8)
    phase = rng.integers(0, 4, size=n_strings, dtype=np.uint8) if with_phase else np.zeros(n_strings, np.uint8)
    return letters, phase


def neel_occupations(rows, cols):
    """Neel-like product state on a rows x cols lattice: site (r, c) holds an
    alpha electron when r + c is even and a beta electron otherwise.
    Returns (alpha_bits, beta_bits) as integers over the sites."""
    a = b = 0
    for r in range(rows):
        for c in range(cols):
            i = r * cols + c
            if (r + c) % 2 == 0:
                a |= 1 << i
            else:
                b |= 1 << i
    return a, b


def random_symplectic(n_strings, n_qubits, seed, pool=None):
    """Random binary symplectic masks: x, z uint64 [n_strings, W] with bits at or
    above n_qubits clear, and uniform Z4 phases.  With ``pool``, rows are drawn
    from ``pool`` distinct random keys (so that duplicates occur)."""
    rng = np.random.default_rng(seed)
    w = max(1, (n_qubits + 63) // 64)
    rows = n_strings if pool is None else pool

    def draw():
        words = rng.integers(0, 2 ** 63, size=(rows, w), dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=(rows, w), dtype=np.uint64)
        for k in range(w):
            top = n_qubits - 64 * k
            if top < 64:
                words[:, k] &= np.uint64((1 << max(top, 0)) - 1)
        return words

    x, z = draw(), draw()
    if pool is not None:
        pick = rng.integers(0, pool, size=n_strings)
        x, z = x[pick], z[pick]
    phase = rng.integers(0, 4, size=n_strings, dtype=np.uint8)
    return np.ascontiguousarray(x), np.ascontiguousarray(z), phase


def pes_integrals(n_orb, r, seed=5001, r_scale=0.3):
    """Spatial integrals along a synthetic potential-energy scan, returned as
    spin-orbital (h1, h2) arrays of ``spin_orbital_integrals``.

    h(R) = h0 + s (R h1 + R^2 h2) and g(R) = g0 + s (R g1 + R^2 g2) with
    s = r_scale, where (h_k, g_k) is ``molecular_integrals(n_orb, seed + k)``
    expressed in the eigenbasis of h0 (orbitals ordered by h0's eigenvalues).
    In that basis the reference that fills the lowest orbitals is the
    one-body ground state of h0, so the scan starts near a mean-field
    solution, as a molecular scan in its Hartree-Fock orbitals does."""
    hs, gs = zip(*(molecular_integrals(n_orb, seed + k) for k in range(3)))
    _, u = np.linalg.eigh(hs[0])
    h = np.zeros((n_orb, n_orb))
    g = np.zeros((n_orb,) * 4)
    for k in range(3):
        f = 1.0 if k == 0 else r_scale * r ** k
        h = h + f * (u.T @ hs[k] @ u)
        g = g + f * np.einsum("pqrs,pi,qj,rk,sl->ijkl", gs[k], u, u, u, u, optimize=True)
    # the rotation keeps the symmetries only up to rounding: give every
    # symmetric pair of h and every 8-fold orbit of g one exact value, so that
    # Pauli strings whose contributions cancel by symmetry cancel exactly
    h = 0.5 * (h + h.T)
    g = g[_orbit_representatives(n_orb)]
    return spin_orbital_integrals(h, g)


def _excitation_qubits(n_orb, n_alpha, n_beta, count, seed):
    """Sorted qubit tuples of the ansatz's excitations, in ansatz order: every
    spin-conserving single (i -> a), then every spin-conserving double
    (i j -> a b) in a seeded random order, cut to ``count``."""
    occ = [p for p in range(n_alpha)] + [n_orb + p for p in range(n_beta)]
    vir = [p for p in range(n_alpha, n_orb)] + [n_orb + p for p in range(n_beta, n_orb)]
    spin = lambda q: q // n_orb
    singles = [(i, a) for i in occ for a in vir if spin(i) == spin(a)]
    doubles = []
    for ii, i in enumerate(occ):
        for j in occ[ii + 1:]:
            for aa, a in enumerate(vir):
                for b in vir[aa + 1:]:
                    if sorted((spin(i), spin(j))) == sorted((spin(a), spin(b))):
                        doubles.append((i, j, a, b))
    rng = np.random.default_rng(seed)
    doubles = [doubles[k] for k in rng.permutation(len(doubles))]
    return [tuple(sorted(q)) for q in (singles + doubles)[:count]]


def excitation_generators(n_orb, n_alpha, n_beta, count, seed=7):
    """Letter strings (uint8 rows over 2 n_orb qubits, 0=I 1=X 2=Y 3=Z) that
    generate the rotations of a synthetic excitation ansatz on the reference
    with the lowest n_alpha alpha and n_beta beta spin-orbitals occupied.

    Every spin-conserving single (i -> a) and double (i j -> a b) excitation
    from occupied to empty spin-orbitals gives one string: Y on its lowest
    qubit, X on its other qubits, and Z on the qubits strictly inside each
    consecutive pair of its sorted qubits (first-second, third-fourth).  The
    list holds all singles, then the doubles in a seeded random order, cut
    to ``count`` strings.  ``excitation_masks`` gives the same strings as
    X/Z bit masks."""
    n = 2 * n_orb
    rows = []
    for qs in _excitation_qubits(n_orb, n_alpha, n_beta, count, seed):
        s = np.zeros(n, np.uint8)
        for a, b in zip(qs[0::2], qs[1::2]):
            s[a + 1:b] = 3
        s[list(qs)] = 1
        s[qs[0]] = 2
        rows.append(s)
    return np.array(rows, dtype=np.uint8).reshape(len(rows), n)


def excitation_masks(n_orb, n_alpha, n_beta, count, seed=7):
    """The strings of ``excitation_generators`` as (x, z) uint64 masks (bit k
    = qubit k), the form the library's rotation ansatz takes: x has every
    qubit of the excitation, z the lowest one (the Y) and the qubits strictly
    inside each consecutive pair."""
    xs, zs = [], []
    for qs in _excitation_qubits(n_orb, n_alpha, n_beta, count, seed):
        xm = 0
        for q in qs:
            xm |= 1 << q
        zm = 1 << qs[0]
        for a, b in zip(qs[0::2], qs[1::2]):
            zm |= ((1 << b) - 1) & ~((1 << (a + 1)) - 1)
        xs.append(xm)
        zs.append(zm)
    x = np.array(xs, dtype=np.uint64)
    return x, np.array(zs, dtype=np.uint64)


def mlp_init(hidden, n_out, seed):
    """Initial parameters of the warm-start network, float32, packed as
    [W1 (H), b1 (H), W2 (H*H), b2 (H), W3 (n_out*H), b3 (n_out)]:
    W1 ~ U(-4, 4), b1 ~ U(-2, 2), W2 ~ U(+-sqrt(3/H)), b2 = 0,
    W3 ~ U(+-0.1 sqrt(3/H)), b3 = 0."""
    rng = np.random.default_rng(seed)
    H, O = hidden, n_out
    a = np.sqrt(3.0 / H)
    parts = [rng.uniform(-4, 4, H), rng.uniform(-2, 2, H), rng.uniform(-a, a, H * H), np.zeros(H),
             rng.uniform(-0.1 * a, 0.1 * a, O * H), np.zeros(O)]
    return np.concatenate(parts).astype(np.float32)


def batched_sector_jobs(n_jobs=64):
    """Uneven sector jobs of the batched workload: job i has n_orb = 10 + i % 4,
    N_e = n_orb + (-2, -1, 0, 1)[(i // 4) % 4] electrons,
    2 S_z = N_e % 2 + 2 ((i // 16) % 2), its own integrals (seed 3000 + i) and
    its own state (seed 3100 + i).  Returns (n_orb, N_alpha, N_beta,
    integral seed, state seed) per job."""
    out = []
    for i in range(n_jobs):
        n_orb = 10 + i % 4
        n_e = n_orb + (-2, -1, 0, 1)[(i // 4) % 4]
        two_sz = n_e % 2 + 2 * ((i // 16) % 2)
        out.append((n_orb, (n_e + two_sz) // 2, (n_e - two_sz) // 2, 3000 + i, 3100 + i))
    return out
