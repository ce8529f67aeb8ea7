"""The compulsory-byte model behind every roofline figure, recomputed from
the storage formats: a link is 9 complex entries (6 with 12-parameter
storage), a colour vector 3 complex, in 8-, 4- or 2-byte reals; fp16 storage
adds one 4-byte scale per vector and one per site for its eight links."""

import pytest

from paper_1111_0125_amd import costs

REAL = {"f64": 8, "f32": 4, "f16s": 2}


def link(prec, r12):
    return (6 if r12 else 9) * 2 * REAL[prec]


def vec(prec):
    return 3 * 2 * REAL[prec] + (4 if prec == "f16s" else 0)


def site_links(prec, r12, nlinks=8):
    return nlinks * link(prec, r12) + (4 if prec == "f16s" else 0)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("r12", [False, True])
@pytest.mark.parametrize("nrhs", [1, 8])
def test_hop_and_A_bytes(prec, r12, nrhs):
    L = site_links(prec, r12)
    v = vec(prec)
    # stage 1: links, read the input, write t; stage 2 also reads the own-site vector
    assert costs.hop_bytes_per_site(prec, 1, nrhs, r12=r12) == L + nrhs * 2 * v
    assert costs.hop_bytes_per_site(prec, 2, nrhs, r12=r12) == L + nrhs * 3 * v
    # inside CG: stage 1 also reads r, stage 2 reads r and writes the new direction
    assert costs.hop_bytes_per_site(prec, 1, nrhs, lazy=True, r12=r12) == L + nrhs * 3 * v
    assert costs.hop_bytes_per_site(prec, 2, nrhs, lazy=True, r12=r12) == L + nrhs * 5 * v
    assert costs.a_bytes_per_site(prec, nrhs, r12=r12) == 2 * L + nrhs * 5 * v


def test_improved_operator_doubles_links_only():
    for prec in ("f64", "f32", "f16s"):
        assert (costs.hop_bytes_per_site(prec, 1, improved=True)
                == site_links(prec, False, 16) + 2 * vec(prec))


def test_update_and_iteration_bytes():
    # fp64 CG: x, r read and written, d and A d read; mixed: y (fp32) read and
    # written, r read and written, d and A d read, in the storage precision
    assert costs.update_bytes_per_site("f64", False) == 6 * vec("f64")
    assert costs.update_bytes_per_site("f32", True) == 2 * vec("f32") + 4 * vec("f32")
    assert costs.update_bytes_per_site("f16s", True) == 2 * vec("f32") + 4 * vec("f16s")
    for prec, mixed in (("f64", False), ("f32", True), ("f16s", True)):
        for r12 in (False, True):
            it = (costs.hop_bytes_per_site(prec, 1, lazy=True, r12=r12)
                  + costs.hop_bytes_per_site(prec, 2, lazy=True, r12=r12)
                  + costs.update_bytes_per_site(prec, mixed))
            assert costs.cg_iteration_bytes_per_site(prec, mixed, r12=r12) == it
    # the figures quoted for the 12-parameter links
    assert [costs.a_bytes_per_site(p, r12=True) for p in ("f64", "f32", "f16s")] == [1776, 888, 472]
    assert [costs.cg_iteration_bytes_per_site(p, p != "f64", r12=True)
            for p in ("f64", "f32", "f16s")] == [2208, 1104, 632]


def test_paper_convention_counts_every_neighbour():
    # Sec.2: 8 links, 8 neighbour vectors and one output per site and D, no reuse
    assert costs.paper_d_bytes_per_site("f64") == (8 * 18 + 8 * 6 + 6) * 8 == 1584
    assert costs.paper_d_bytes_per_site("f32", r12=True) == (8 * 12 + 8 * 6 + 6) * 4
    assert costs.a_flops_per_site() == 2 * 576 + 12
