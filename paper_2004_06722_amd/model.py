"""Algorithmic byte and flop counts of the bake-off hot path.

Bytes are what the method itself must move per CG iteration: the stored
geometric factors (section 5 after eq. (gij): 6 q^3 words per element for the
stiffness, q^3 for B~ of eq. (mass)), the int32 gather map (p1^3 per element;
the global tensor layout may not be exploited, section 3), and the vectors.
Vector words per DOF and iteration: the operator reads p and writes w (2),
the CG updates move 10 with the preconditioned residual z = D^-1 r kept in
place of r: the residual update reads z, w, dinv and writes z and the zeroed
w for the next scatter (5), the solution and direction update reads x, p, z
and writes x, p (5). 12 in all. DOFs are n = p^3 E (section 2) per component.

Flops follow section 5: eq. (work2)/(work3) for the sum-factorised
stiffness, 4 p1^4 (g^3 + g^2 + g) for the mass, with J^ = I for collocated
GLL (the derivative contractions alone: 12 p1^4 + 15 p1^3).
"""
from __future__ import annotations

VECTOR_WORDS_OPERATOR = 2
VECTOR_WORDS_CG = 10


def points(p: int, E: int) -> int:
    """n = p^3 E, the point count of section 2 (no boundary or redundancy
    effects): the n of every DOFs/s figure."""
    return p ** 3 * E


def quadrature(bp: int, p: int) -> int:
    return p + 1 if bp in (5, 6) else p + 2


def geometry_words(bp: int, p: int) -> int:
    q = quadrature(bp, p)
    return (6 if bp >= 3 else 1) * q ** 3


def apply_bytes(bp: int, p: int, E: int, ncomp: int = 1, word: int = 8) -> int:
    """Bytes of one operator application (geometry + map + u in + w out)."""
    n = p ** 3 * E
    return E * (word * geometry_words(bp, p) + 4 * (p + 1) ** 3) \
        + word * VECTOR_WORDS_OPERATOR * n * ncomp


def mass_element_bytes(p: int, E: int, ncomp: int = 1, word: int = 8) -> int:
    """Bytes of the Gauss-Legendre mass kernel as the PCG runs it for BP1/BP2:
    B~ + map + u gathered (one word per DOF) + w_L stored per element
    ((p+1)^3 words per element and component). The assembly Q^T w_L is done by
    the residual update, so these are the bytes of the timed operator launch;
    the iteration counts keep the algorithmic operator bytes of apply_bytes."""
    return E * (word * geometry_words(1, p) + 4 * (p + 1) ** 3) \
        + word * ncomp * (p ** 3 * E + E * (p + 1) ** 3)


def helm_apply_bytes(bp: int, p: int, E: int, ncomp: int = 1, word: int = 8) -> int:
    """Bytes of one Helmholtz application H = A + B_beta (eq. (hm2)) read once:
    the stiffness application plus beta B~ (q^3 words per element)."""
    return apply_bytes(bp, p, E, ncomp, word) + E * word * quadrature(bp, p) ** 3


def local_apply_bytes(bp: int, p: int, E: int, ncomp: int = 1, word: int = 8) -> int:
    """Bytes of one unassembled application w_L = A_L u_L (the BK kernels):
    geometry + element-local u_L in + w_L out, (p+1)^3 words each per element
    and component; no gather map."""
    return E * (word * geometry_words(bp, p) + 2 * word * ncomp * (p + 1) ** 3)


def iteration_bytes(bp: int, p: int, E: int, ncomp: int = 1, word: int = 8,
                    interior_order: bool = True) -> int:
    """Bytes of one CG iteration (operator + vector updates). With the
    library's internal node order (the default) the residual update does not
    clear w on the (p-1)^3 element-interior nodes of each element, which the
    operator overwrites with plain stores: one word less there. The Gauss-
    Legendre mass (BP1/BP2) assembles by a gather and has no w to clear. The
    inverse diagonal is read once per node for all components."""
    n = p ** 3 * E
    # dinv (one of the ten words) is shared by the components
    b = apply_bytes(bp, p, E, ncomp, word) + word * ((VECTOR_WORDS_CG - 1) * ncomp + 1) * n
    if interior_order and bp >= 3:
        b -= word * max(p - 1, 0) ** 3 * E * ncomp
    return b


def work_direct(p1: int, gamma: float) -> float:
    """Eq. (work2): D_j applied in factored form, (J^ x J^ x D^) per direction."""
    return 4 * p1 ** 4 * (3 * gamma ** 3 + 3 * gamma ** 2 + 2 * gamma) + 15 * gamma ** 3 * p1 ** 3


def work_interpolate_first(p1: int, gamma: float) -> float:
    """Eq. (work3): interpolate to the quadrature points, differentiate there."""
    return 4 * p1 ** 4 * (3 * gamma ** 4 + gamma ** 3 + gamma ** 2 + gamma) \
        + 15 * gamma ** 3 * p1 ** 3


def work_mass(p1: int, gamma: float) -> float:
    """Section 5 after eq. (mass): 4 p1^4 (g^3 + g^2 + g) (+ q^3 for B~)."""
    return 4 * p1 ** 4 * (gamma ** 3 + gamma ** 2 + gamma) + (gamma * p1) ** 3


def apply_flops_per_element(bp: int, p: int) -> float:
    p1 = p + 1
    q = quadrature(bp, p)
    g = q / p1
    if bp in (5, 6):
        return 12 * p1 ** 4 + 15 * p1 ** 3      # J^ = I: only the D^ contractions
    if bp in (3, 4):
        return work_interpolate_first(p1, g)
    return work_mass(p1, g)


def iteration_flops(bp: int, p: int, E: int, ncomp: int = 1) -> float:
    """Operator flops + 12 flops per DOF for the CG vector updates and dots."""
    n = p ** 3 * E
    return (apply_flops_per_element(bp, p) * E + 12 * n) * ncomp


HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published
FP32_PEAK_TFLOPS = 157.3
