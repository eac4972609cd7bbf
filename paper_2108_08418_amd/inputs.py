"""Seeded synthetic inputs shared by the fp64 oracle and the HIP path.

This module holds no step of the reconciliation method itself.  It builds
only what the method consumes:

* parity-check matrices H (Tanner graphs) -- the codes the paper leaves to a
  private database (Sec. V-B) are replaced by seeded constructions here;
* Alice/Bob quadrature pairs of the AWGN channel used in the experiments
  (Sec. V: x ~ N(0, V_A), y = x + n, n ~ N(0, sigma_n^2), gamma = 1/sigma_n^2);
* BPSK-over-AWGN channel LLRs (2y/sigma^2) for the plain decoder workloads;
* quantiser thresholds (the quantiser M(.) of Sec. III-B takes them as
  parameters; equiprobable thresholds are one admissible choice).

Every generator takes an explicit seed and uses NumPy's PCG64 so that both
sides of a parity test see byte-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.special import ndtri

__all__ = [
    "CsrCode", "QcCode", "largest_remainder", "regular_code", "irregular_code",
    "qc_protograph_code", "gaussian_pairs", "bpsk_llr", "random_bits",
    "equiprobable_thresholds", "LAMBDA_NODE_FRACTIONS", "slice_code_spec", "SLICE_MB",
    "met_low_rate_spec", "lambda_half_rate_spec", "slice_code_at",
]

# lambda(x) = 0.25 x + 0.3 x^2 + 0.45 x^7 (edge perspective).  Node-perspective
# fractions are lambda_a/a normalised: (0.125, 0.1, 0.05625)/0.28125.
LAMBDA_EDGE = {2: 0.25, 3: 0.30, 8: 0.45}
LAMBDA_NODE_FRACTIONS = {
    d: (lam / d) / sum(l / k for k, l in LAMBDA_EDGE.items()) for d, lam in LAMBDA_EDGE.items()
}


def largest_remainder(fracs, total: int) -> np.ndarray:
    """Integer counts summing to ``total`` closest to ``fracs * total``."""
    fr = np.asarray(fracs, dtype=np.float64)
    raw = fr / fr.sum() * total
    base = np.floor(raw).astype(np.int64)
    short = int(total - base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:short]] += 1
    return base


@dataclass
class CsrCode:
    """Sparse H with ``m`` rows (checks) and ``n`` columns (variables).

    Row ``c`` holds columns ``col_idx[row_ptr[c]:row_ptr[c+1]]`` in ascending
    order.  ``edge_type[e]`` is the edge class used by per-type min-sum weights.
    """
    n: int
    m: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    edge_type: np.ndarray
    n_types: int = 1
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        h = np.zeros((self.m, self.n), dtype=np.uint8)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        h[rows, self.col_idx] = 1
        return h

    def var_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.n)

    def check_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


@dataclass
class QcCode:
    """Quasi-cyclic H lifted from an ``mb x nb`` protograph by ``Z x Z`` circulants.

    ``shift[i, j] = -1`` marks a zero block.  Otherwise block (i, j) is the
    identity cyclically shifted so that check ``i*Z + k`` is connected to
    variable ``j*Z + (k + shift[i, j]) mod Z``.
    """
    nb: int
    mb: int
    Z: int
    shift: np.ndarray            # int32 [mb, nb]
    block_type: np.ndarray       # uint8 [mb, nb]
    n_types: int = 1
    name: str = ""

    @property
    def n(self) -> int:
        return self.nb * self.Z

    @property
    def m(self) -> int:
        return self.mb * self.Z

    @property
    def n_edges(self) -> int:
        return int((self.shift >= 0).sum()) * self.Z

    def to_csr(self) -> CsrCode:
        """Expand to an explicit CSR matrix (columns ascending within a row)."""
        Z = self.Z
        k = np.arange(Z, dtype=np.int64)
        per_row_cols = []
        per_row_types = []
        for i in range(self.mb):
            js = np.nonzero(self.shift[i] >= 0)[0]
            # [deg, Z] column index for every check k of block row i
            c = np.stack([j * Z + (k + self.shift[i, j]) % Z for j in js]) if len(js) else np.zeros((0, Z), np.int64)
            t = np.repeat(self.block_type[i, js][:, None], Z, axis=1) if len(js) else np.zeros((0, Z), np.uint8)
            per_row_cols.append(c.T)   # [Z, deg]; js ascending -> columns ascending
            per_row_types.append(t.T)
        col_idx = np.concatenate([c.reshape(-1) for c in per_row_cols]).astype(np.int32)
        edge_type = np.concatenate([t.reshape(-1) for t in per_row_types]).astype(np.uint8)
        degs = np.concatenate([np.full(Z, c.shape[1], dtype=np.int64) for c in per_row_cols])
        row_ptr = np.zeros(self.m + 1, dtype=np.int32)
        np.cumsum(degs, out=row_ptr[1:])
        return CsrCode(self.n, self.m, row_ptr, col_idx, edge_type, self.n_types, self.name + "/csr")


def _match_sockets(vdeg: np.ndarray, cdeg: np.ndarray, rng: np.random.Generator):
    """Configuration model without repeated (v, c) pairs.

    Variable sockets are permuted at random against check sockets taken in
    order; each repeated pair is then removed by swapping its variable endpoint
    with that of a uniformly drawn edge, when the swap creates no new repeat.
    Both degree sequences are preserved exactly.
    """
    vs = np.repeat(np.arange(len(vdeg), dtype=np.int64), vdeg)
    cs = np.repeat(np.arange(len(cdeg), dtype=np.int64), cdeg)
    if len(vs) != len(cs):
        raise ValueError("socket counts differ")
    vs = vs[rng.permutation(len(vs))]
    m = len(cdeg)
    keys = vs * m + cs
    counts: dict[int, int] = {}
    for kk in keys.tolist():
        counts[kk] = counts.get(kk, 0) + 1
    dups = [e for e in range(len(keys)) if counts[int(keys[e])] > 1]
    guard = 0
    while dups:
        guard += 1
        if guard > 1_000_000:
            raise RuntimeError("could not remove repeated edges")
        e = dups.pop()
        ke = int(vs[e] * m + cs[e])
        if counts.get(ke, 0) <= 1:
            continue
        e2 = int(rng.integers(len(vs)))
        if e2 == e:
            dups.append(e)
            continue
        a = int(vs[e2] * m + cs[e])     # new pair for edge e
        b = int(vs[e] * m + cs[e2])     # new pair for edge e2
        if a == b or counts.get(a, 0) or counts.get(b, 0):
            dups.append(e)
            continue
        k2 = int(vs[e2] * m + cs[e2])
        counts[ke] -= 1
        counts[k2] -= 1
        counts[a] = 1
        counts[b] = 1
        vs[e], vs[e2] = vs[e2], vs[e]
    return vs, cs


def _csr_from_edges(n, m, vs, cs, edge_type_of_var=None, n_types=1, name=""):
    order = np.lexsort((vs, cs))
    vs = vs[order]
    cs = cs[order]
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(np.bincount(cs, minlength=m), out=row_ptr[1:])
    col_idx = vs.astype(np.int32)
    if edge_type_of_var is None:
        et = np.zeros(len(vs), dtype=np.uint8)
    else:
        et = np.asarray(edge_type_of_var, dtype=np.uint8)[vs]
    return CsrCode(n, m, row_ptr, col_idx, et, n_types, name)


def regular_code(n: int, dv: int, dc: int, seed: int) -> CsrCode:
    """(dv, dc)-regular H from a seeded edge permutation with no repeated edges."""
    if (n * dv) % dc:
        raise ValueError("n*dv must be divisible by dc")
    m = n * dv // dc
    rng = np.random.default_rng(seed)
    vs, cs = _match_sockets(np.full(n, dv), np.full(m, dc), rng)
    return _csr_from_edges(n, m, vs, cs, name=f"reg({dv},{dc})n{n}s{seed}")


def _var_degree_sequence(n, node_fracs: dict[int, float]):
    degs = sorted(node_fracs)
    counts = largest_remainder([node_fracs[d] for d in degs], n)
    vdeg = np.repeat(np.array(degs, dtype=np.int64), counts)
    vtype = np.repeat(np.arange(len(degs), dtype=np.uint8), counts)
    return vdeg, vtype


def _concentrated_checks(E: int, m: int) -> np.ndarray:
    lo = E // m
    n_hi = E - lo * m
    return np.concatenate([np.full(m - n_hi, lo, dtype=np.int64), np.full(n_hi, lo + 1, dtype=np.int64)])


def irregular_code(n: int, m: int, node_fracs: dict[int, float], seed: int) -> CsrCode:
    """Irregular H: variable degrees from node fractions (largest remainder),
    check degrees concentrated on floor/ceil(E/m).  Edge type = variable degree class.
    """
    rng = np.random.default_rng(seed)
    vdeg, vtype = _var_degree_sequence(n, node_fracs)
    perm = rng.permutation(n)          # spread degree classes over column positions
    vdeg, vtype = vdeg[perm], vtype[perm]
    E = int(vdeg.sum())
    cdeg = _concentrated_checks(E, m)
    cdeg = cdeg[rng.permutation(m)]
    vs, cs = _match_sockets(vdeg, cdeg, rng)
    return _csr_from_edges(n, m, vs, cs, vtype, len(node_fracs), name=f"irr n{n} m{m} s{seed}")


def _assign_shifts(base: np.ndarray, Z: int, rng: np.random.Generator, tries: int = 64) -> np.ndarray:
    """Circulant shifts in [0, Z), redrawn (up to ``tries`` times) while they
    close a length-4 cycle with shifts already drawn."""
    mb, nb = base.shape
    shift = np.full((mb, nb), -1, dtype=np.int64)
    rows_of = [np.nonzero(base[:, j])[0] for j in range(nb)]
    for i in range(mb):
        for j in np.nonzero(base[i])[0]:
            best = None
            for _ in range(tries):
                s = int(rng.integers(Z))
                bad = False
                for j2 in np.nonzero(shift[i] >= 0)[0]:
                    for i2 in rows_of[j]:
                        if i2 == i or shift[i2, j] < 0 or shift[i2, j2] < 0:
                            continue
                        if (s - shift[i, j2] + shift[i2, j2] - shift[i2, j]) % Z == 0:
                            bad = True
                            break
                    if bad:
                        break
                best = s
                if not bad:
                    break
            shift[i, j] = best
    return shift


def qc_protograph_code(nb: int, mb: int, Z: int, col_degrees: np.ndarray, seed: int,
                       col_type: np.ndarray | None = None, n_types: int | None = None,
                       name: str = "") -> QcCode:
    """QC-LDPC code: a seeded ``mb x nb`` binary protograph with the given column
    degrees and concentrated row degrees, lifted by seeded circulants of size Z."""
    rng = np.random.default_rng(seed)
    col_degrees = np.asarray(col_degrees, dtype=np.int64)
    if col_degrees.max() > mb:
        raise ValueError("column degree exceeds number of block rows")
    E = int(col_degrees.sum())
    rdeg = _concentrated_checks(E, mb)[rng.permutation(mb)]
    vs, cs = _match_sockets(col_degrees, rdeg, rng)
    base = np.zeros((mb, nb), dtype=np.uint8)
    base[cs, vs] = 1
    shift = _assign_shifts(base, Z, rng)
    if col_type is None:
        col_type = np.zeros(nb, dtype=np.uint8)
        n_types = 1
    btype = np.where(shift >= 0, np.asarray(col_type, dtype=np.uint8)[None, :], 0).astype(np.uint8)
    return QcCode(nb, mb, Z, shift.astype(np.int32), btype, int(n_types), name)


def _lambda_columns(nb: int):
    degs = sorted(LAMBDA_NODE_FRACTIONS)
    counts = largest_remainder([LAMBDA_NODE_FRACTIONS[d] for d in degs], nb)
    col_deg = np.repeat(np.array(degs), counts)
    col_type = np.repeat(np.arange(len(degs), dtype=np.uint8), counts)
    return col_deg, col_type


def _chain_base_matrix(col_deg: np.ndarray, mb: int, rng: np.random.Generator) -> np.ndarray:
    """Binary protograph whose degree-2 columns form one path through the rows
    (so no cycle runs through degree-2 columns only: such cycles lift to
    low-weight codewords), the other columns filling the least-loaded rows.
    Row order and tie-breaking are seeded."""
    nb = len(col_deg)
    base = np.zeros((mb, nb), dtype=np.uint8)
    rows = rng.permutation(mb)
    d2 = np.nonzero(col_deg == 2)[0]
    if len(d2) >= mb:
        raise ValueError("too many degree-2 columns for an acyclic chain")
    for k, c in enumerate(d2):
        base[rows[k], c] = 1
        base[rows[k + 1], c] = 1
    for c in np.nonzero(col_deg != 2)[0]:
        load = base.sum(1) + rng.random(mb) * 0.5
        base[np.argsort(load, kind="stable")[: col_deg[c]], c] = 1
    return base


def layer_order(base: np.ndarray, group: int = 8) -> np.ndarray:
    """An order of the block rows of a protograph in runs of at most ``group``
    rows that pairwise share no block column.  Rows of such a run touch
    disjoint variables, so a layered decoder may update them together; the
    order only lists the same checks differently.  Greedy: each run takes the
    remaining rows in order of most column conflicts with the other remaining
    rows (ties by index) that conflict with none already in the run."""
    mb = base.shape[0]
    b = (base != 0).astype(np.int64)
    conflict = (b @ b.T) > 0
    np.fill_diagonal(conflict, False)
    left = list(range(mb))
    order = []
    while left:
        run = []
        for r in sorted(left, key=lambda r: (-int(conflict[r, left].sum()), r)):
            if len(run) == group:
                break
            if not any(conflict[r, q] for q in run):
                run.append(r)
        for r in run:
            left.remove(r)
        order.extend(run)
    return np.asarray(order, dtype=np.int64)


def _lambda_qc_code(nb: int, mb: int, Z: int, seed: int, name: str) -> QcCode:
    """The protograph depends on ``seed`` only, so that every lifting size Z
    shares it (and per-edge-type decoder weights carry over between sub-block
    lengths); the circulant shifts depend on (seed, Z).  Block rows are listed
    in ``layer_order``: runs of up to 8 rows with disjoint columns, the layers
    a layered schedule updates together."""
    col_deg, col_type = _lambda_columns(nb)
    rng = np.random.default_rng(seed)
    p = rng.permutation(nb)
    col_deg, col_type = col_deg[p], col_type[p]
    base = _chain_base_matrix(col_deg, mb, rng)
    shift = _assign_shifts(base, Z, np.random.default_rng([seed, Z]))
    shift = shift[layer_order(base)]
    btype = np.where(shift >= 0, col_type[None, :], 0).astype(np.uint8)
    return QcCode(nb, mb, Z, shift.astype(np.int32), btype, 3, name=name)


# Block rows (of nb = 128) of the coded slices' codes, as the rate-selection
# loop of Sec. V-B picks them (rates.select_slice_rate with 256 test
# sub-blocks of n = 65536 on the GPU path): start 10 % below the slice
# capacity and step down by 0.05 while a test sub-block fails.
#   slice 2 (C = 0.3156): R = 0.2813 fails 256/256, 0.2344 fails 91/256,
#                         0.1875 (mb = 104) fails none;
#   slice 3 (C = 0.5468): R = 0.4922 (mb = 65) fails none.
SLICE_MB = {2: 104, 3: 65}


def slice_code_spec(slice_j: int, n: int, seed: int = 2108) -> QcCode:
    """Seeded QC code for coded slice ``slice_j`` (2 or 3) of the 16-level,
    4-slice setup at SNR 3: lambda(x) = 0.25x + 0.3x^2 + 0.45x^7 over nb = 128
    block columns, degree-2 columns chained (see ``_chain_base_matrix``), at
    the rate the selection loop picks (``SLICE_MB``): slice 2 R = 0.1875,
    slice 3 R = 0.4921875.  Column permutation and shifts are seeded; block
    rows are listed in ``layer_order``."""
    return slice_code_at(slice_j, n, SLICE_MB[slice_j], seed)


def slice_code_at(slice_j: int, n: int, mb: int, seed: int = 2108) -> QcCode:
    """The slice-``slice_j`` code family at mb of the nb = 128 block rows
    (rate 1 - mb/128): the candidates of the rate-selection loop."""
    nb = 128
    if n % nb:
        raise ValueError("n must be a multiple of 128")
    if not 0 < mb < nb:
        raise ValueError("mb must be in (0, 128)")
    return _lambda_qc_code(nb, mb, n // nb, seed * 131 + slice_j * 7, f"slice{slice_j}-qc n{n}")


def lambda_half_rate_spec(n: int, seed: int = 1650) -> QcCode:
    """Rate-1/2 QC code with the lambda(x) degree profile (nb = 128, mb = 64)."""
    nb, mb = 128, 64
    if n % nb:
        raise ValueError("n must be a multiple of 128")
    return _lambda_qc_code(nb, mb, n // nb, seed, f"lambda-r1/2-qc n{n}")


def met_low_rate_spec(n: int, seed: int = 16) -> QcCode:
    """Seeded raptor-like multi-edge-type protograph for SNR 0.16, nb = 64.

    Core: 16 columns of degree 3 over 12 core rows.  Extension: 48 rows, each
    with a private degree-1 column and one (24 rows: a repetition observation
    of a core bit) or two (24 rows: a parity of two core bits) core columns,
    spread evenly over the core.  Rate (16 - 12) / 64 = 0.0625.  Edge types:
    0 = core checks, 1 = extension checks to the core, 2 = degree-1 edges.
    Block rows are listed in ``layer_order`` (9 runs of column-disjoint rows).
    Rates 5/64 and 6/64 of this family did not decode at SNR 0.16 (n = 16384),
    4/64 did (no failure in 16 frames).  The protograph
    depends on ``seed`` only, the circulant shifts on (seed, Z).
    """
    nb, n_core, mc = 64, 16, 12
    if n % nb:
        raise ValueError("n must be a multiple of 64")
    Z = n // nb
    rng = np.random.default_rng(seed)
    n_ext = nb - n_core
    mb = mc + n_ext
    base = np.zeros((mb, nb), dtype=np.uint8)
    btype = np.zeros((mb, nb), dtype=np.uint8)
    for j in range(n_core):
        load = base[:mc].sum(1) + rng.random(mc) * 0.5
        base[np.argsort(load, kind="stable")[:3], j] = 1
    for r in range(n_ext):
        k = 1 if r < n_ext // 2 else 2
        cl = base[:, :n_core].sum(0) + rng.random(n_core) * 0.5
        js = np.argsort(cl, kind="stable")[:k]
        base[mc + r, js] = 1
        btype[mc + r, js] = 1
        base[mc + r, n_core + r] = 1
        btype[mc + r, n_core + r] = 2
    shift = _assign_shifts(base, Z, np.random.default_rng([seed, Z]))
    order = layer_order(base)
    shift, btype = shift[order], btype[order]
    btype = np.where(shift >= 0, btype, 0).astype(np.uint8)
    return QcCode(nb, mb, Z, shift.astype(np.int32), btype, 3, name=f"met-r0.0625-qc n{n}")


# ----------------------------------------------------------------------------
# channel data
# ----------------------------------------------------------------------------

def gaussian_pairs(N: int, snr: float, seed: int):
    """Alice's x ~ N(0, 1) and Bob's y = x + n with n ~ N(0, 1/snr) (Sec. V),
    unit-variance modulation so that SNR = Var X / Var N."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N)
    y = x + rng.standard_normal(N) * np.sqrt(1.0 / snr)
    return x, y


def random_bits(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 2, size=shape, dtype=np.uint8)


def bpsk_llr(bits: np.ndarray, sigma2, seed: int) -> np.ndarray:
    """Channel LLRs ln P(0|y)/P(1|y) = 2y/sigma^2 for BPSK (0 -> +1) over AWGN.

    ``sigma2`` is a scalar or one value per frame (leading axis of ``bits``)."""
    rng = np.random.default_rng(seed)
    s2 = np.asarray(sigma2, dtype=np.float64)
    if s2.ndim == 1:
        s2 = s2.reshape((-1,) + (1,) * (bits.ndim - 1))
    y = (1.0 - 2.0 * bits.astype(np.float64)) + rng.standard_normal(bits.shape) * np.sqrt(s2)
    return 2.0 * y / s2


def sigma2_from_ebn0(ebn0_db, rate: float):
    return 1.0 / (2.0 * rate * 10.0 ** (np.asarray(ebn0_db, dtype=np.float64) / 10.0))


def equiprobable_thresholds(m_bits: int, var_y: float) -> np.ndarray:
    """t_i = sigma_Y * Phi^{-1}(i / 2^m), i = 1..2^m-1, for Y ~ N(0, var_y)."""
    q = np.arange(1, 2 ** m_bits, dtype=np.float64) / 2.0 ** m_bits
    return np.sqrt(var_y) * ndtri(q)


def constant_step_thresholds(m_bits: int, delta: float) -> np.ndarray:
    """t_i = (i - 2^(m-1)) * delta: 2^m equal bins centred on zero (Sec. III-B)."""
    i = np.arange(1, 2 ** m_bits, dtype=np.float64)
    return (i - 2 ** (m_bits - 1)) * delta


@dataclass
class Workload:
    """A named synthetic workload (sizes only; data comes from the generators)."""
    name: str
    params: dict = field(default_factory=dict)
