"""The persistent launch-shape table (STAG_TUNE_CACHE): a context's
stag_tune times the shapes once and appends the result; a later context
(another process would do the same) loads it without timing anything."""

import pytest

from tests.gpu_common import links

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


def test_tune_table_round_trip(stag, tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("STAG_TUNE_CACHE", str(path))
    L = (8, 8, 8, 8)
    U = links(L, "haar", 3)
    with stag.Context(0) as c1:
        g = c1.gauge(L, U, precisions=("f64", "f32"), r12=True)
        cfg1, ms1 = stag.stag_tune(c1, g, "f32", 1)
        assert stag.stag_tune_counts(c1) == (0, 1)
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].split()[1:6] == ["4", "1", str(g.vh), "1", "1"]
    with stag.Context(0) as c2:
        g = c2.gauge(L, U, precisions=("f64", "f32"), r12=True)
        cfg2, ms2 = stag.stag_tune(c2, g, "f32", 1)
        assert stag.stag_tune_counts(c2) == (1, 0)
        assert cfg2 == cfg1 and abs(ms2 - ms1) <= 1e-7 * ms1
        assert stag.stag_tune_get(c2, "f32", 1, g.vh) == cfg1
        # another key (full links) is measured and appended
        g2 = c2.gauge(L, U, precisions=("f64", "f32"))
        stag.stag_tune(c2, g2, "f32", 1)
        assert stag.stag_tune_counts(c2) == (1, 1)
        assert len(path.read_text().splitlines()) == 2
