"""The autotuner's result table on the GPU: a timed result is stored under
its key, reused without timing by a later call (also after a save, clear
and load through the JSON file), forced timing replaces it, and a stored
choice that is not a candidate for the problem is ignored.  The field after
applying a cached choice is bitwise the one after applying the timed choice
(the choice fixes the kernel and its summation order)."""
import numpy as np
import pytest

from gpu_helpers import build, close, device_state, tilemag
from paper_2107_05364_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_tune_results_are_cached_and_reloaded(tmp_path):
    tmg = tilemag()
    ctx = tmg.Context(0)
    c, s = W.grid(30, 10, 1, 5e-9, 5e-9, 3e-9)
    m = device_state(W.random_unit_vectors(5, c.shape[0])[None])
    tmg.tm_tune_cache_clear()
    for layout in (tmg.TM_LAYOUT_SYM6, tmg.TM_LAYOUT_PSYM4):
        g, T, p = build(tmg, ctx, c, s, layout=layout)
        n0 = tmg.tm_tune_cache_size()
        chosen, ms = tmg.tm_problem_tune(p.handle, 1, -3)  # timed
        assert tmg.tm_tune_cache_size() == n0 + 1 and ms > 0
        H = p.heff(m).cpu().numpy()
        # a second problem of the same key takes the stored result, untimed
        g2, T2, p2 = build(tmg, ctx, c, s, layout=layout)
        again, ms2 = tmg.tm_problem_tune(p2.handle, 1, 3)
        assert (again, ms2) == (chosen, ms)
        assert np.array_equal(p2.heff(m).cpu().numpy(), H)
        close(g2, T2, p2)
        close(g, T, p)
    path = tmp_path / "tune.json"
    tmg.tm_tune_cache_save(str(path))
    text = path.read_text()
    tmg.tm_tune_cache_clear()
    assert tmg.tm_tune_cache_size() == 0
    assert tmg.tm_tune_cache_load(str(path)) == tmg.TM_OK and tmg.tm_tune_cache_size() == 2
    g, T, p = build(tmg, ctx, c, s, layout=tmg.TM_LAYOUT_PSYM4)
    loaded, ms3 = tmg.tm_problem_tune(p.handle, 1, 3)
    assert '"choice": %d' % loaded in text and ms3 > 0
    # a stored choice that is no candidate (loads are 0 or 1) is not applied: the call times
    bogus = text.replace('"layout": 4, "prec": 0, "n": 300, "batch": 1, "choice": %d' % loaded,
                         '"layout": 4, "prec": 0, "n": 300, "batch": 1, "choice": 7')
    assert bogus != text
    path.write_text(bogus)
    tmg.tm_tune_cache_clear()
    tmg.tm_tune_cache_load(str(path))
    chosen, ms4 = tmg.tm_problem_tune(p.handle, 1, 3)
    assert chosen in (0, 1)
    close(g, T, p)
    tmg.tm_tune_cache_clear()
    ctx.close()


def test_apply_reproduces_a_choice():
    """tm_problem_apply sets what tm_problem_tune would choose, untimed: the
    pair-symmetric loads (the field is the same either way), a SYM6 launch
    shape (tm_problem_shape reports it); a non-candidate is refused and
    changes nothing."""
    tmg = tilemag()
    ctx = tmg.Context(0)
    c, s = W.grid(30, 10, 1, 5e-9, 5e-9, 3e-9)
    m = device_state(W.random_unit_vectors(7, c.shape[0])[None])
    g, T, p = build(tmg, ctx, c, s, layout=tmg.TM_LAYOUT_PSYM4)
    fields = []
    for choice in (0, 1):
        tmg.tm_problem_apply(p.handle, choice)
        fields.append(p.heff(m).cpu().numpy())
    assert np.array_equal(fields[0], fields[1])
    with pytest.raises(tmg.TilemagError):
        tmg.tm_problem_apply(p.handle, 2)
    close(g, T, p)
    g, T, p = build(tmg, ctx, c, s, layout=tmg.TM_LAYOUT_SYM6)
    for shape in (3, tmg.tm_num_shapes() - 1):
        tmg.tm_problem_apply(p.handle, shape)
        assert tmg.tm_problem_shape(p.handle) == shape
    with pytest.raises(tmg.TilemagError):
        tmg.tm_problem_apply(p.handle, tmg.tm_num_shapes())
    assert tmg.tm_problem_shape(p.handle) == tmg.tm_num_shapes() - 1
    close(g, T, p)
    ctx.close()
