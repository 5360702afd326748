"""Pins of the algorithmic byte and flop counts that bench.py divides by the
measured times (the roofline fractions): per-element figures of section 5
worked out by hand at N = 7."""
import pytest

from paper_2004_06722_amd import model


def test_bk5_per_element_counts_at_n7():
    # collocated GLL, q = p1 = 8: six G words per point (eq. (gij)), 512 points
    assert model.geometry_words(5, 7) == 6 * 512
    # J^ = I: three derivative contractions and their transposes,
    # 6 x 2 p1^4, plus 15 flops per point for G (u_r, u_s, u_t)
    assert model.apply_flops_per_element(5, 7) == 12 * 8 ** 4 + 15 * 8 ** 3 == 56832
    # one element's operator: 24,576 B of G + 2,048 B of int32 map + u in,
    # w out (two words per DOF, 343 DOFs per element)
    assert model.apply_bytes(5, 7, 1) == 24576 + 2048 + 2 * 8 * 343
    # a PCG iteration adds ten vector words per DOF, less the clearing of w on
    # the 216 element-interior nodes in the internal node order
    assert model.iteration_bytes(5, 7, 1, interior_order=False) == \
        model.apply_bytes(5, 7, 1) + 10 * 8 * 343
    assert model.iteration_bytes(5, 7, 1) == model.apply_bytes(5, 7, 1) + 10 * 8 * 343 - 8 * 216


def test_bp1_counts_at_n7():
    # Gauss-Legendre q = p + 2 = 9: one B~ word per point (eq. (mass))
    assert model.geometry_words(1, 7) == 9 ** 3
    assert model.apply_bytes(1, 7, 1) == 8 * 729 + 4 * 512 + 2 * 8 * 343
    # the mass kernel as the PCG runs it: u gathered (343 words), w_L stored
    # per element slot (512 words) instead of w scatter-added
    assert model.mass_element_bytes(7, 1) == 8 * 729 + 4 * 512 + 8 * (343 + 512) == 14720
    assert model.mass_element_bytes(7, 10, ncomp=3) == \
        10 * (8 * 729 + 4 * 512) + 3 * 8 * 10 * (343 + 512)


@pytest.mark.parametrize("p", [1, 3, 8])
def test_mass_flops_reduce_to_the_tensor_form(p):
    # 4 p1^4 (g^3 + g^2 + g) + q^3 with g = q / p1: the J^ chain there and
    # back (three contractions each way, 2 flops per multiply-add) and B~
    p1, q = p + 1, p + 2
    chain = 2 * 2 * (q * p1 ** 3 + q * q * p1 ** 2 + q ** 3 * p1)
    assert model.apply_flops_per_element(1, p) == pytest.approx(chain + q ** 3)


def _paper_counts():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")
    with open(path) as f:
        return json.load(f)


def test_point_count_matches_the_paper_example():
    # section 2: p = 7 with E = 2^14 and 2^16 gives the printed n
    for row in _paper_counts()["n_points"]:
        assert model.points(row["p"], row["E"]) == row["n"]


@pytest.mark.parametrize("row", _paper_counts()["interpolate_first"])
def test_interpolate_first_relative_work_matches_the_paper(row):
    # section 5 after eq. (work3): interpolating to the quadrature points first
    # changes the work of eq. (work2) by about -25% at gamma = 1 and +12% at
    # gamma = 3/2 (leading order: large p1, where the p1^3 term is small)
    p1, g = row["p1_large"], row["gamma"]
    change = model.work_interpolate_first(p1, g) / model.work_direct(p1, g) - 1.0
    assert abs(change - row["relative_change"]) <= row["tolerance"], change


def test_vector_iteration_counts_dinv_once():
    # three components share the map, G and the inverse diagonal: nine vector
    # words per component and DOF plus one for dinv
    E, n = 1, 343
    assert model.iteration_bytes(6, 7, E, 3, interior_order=False) == \
        model.apply_bytes(6, 7, E, 3) + 8 * (9 * 3 + 1) * n
