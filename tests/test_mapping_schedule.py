"""Host logic of the mapping loop's schedules (no GPU: the Mapper's buffers are built only
when an item first runs)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _mapper(schedule, iterations=90):
    from paper_2412_01217_amd import mapping, raster, scenes
    views = [scenes.identity_view(64, 48, levels=3), scenes.identity_view(64, 48, levels=3)]
    cfg = raster.config(4)
    n = 10
    g = dict(mean=torch.zeros(n, 3), log_scale=torch.zeros(n, 3), quat=torch.zeros(n, 4), opacity=torch.zeros(n),
             rgb=torch.zeros(n, 3), sem=torch.zeros(n, 4))
    return mapping.Mapper(cfg, g, views, targets={}, n_classes=4, schedule=schedule, iterations=iterations, seed=1)


def test_random_schedule_draws_every_keyframe_and_level():
    mp = _mapper("random")
    keys = [mp.draw(i) for i in range(400)]
    assert set(keys) == {(k, l) for k in range(2) for l in range(3)}
    counts = np.bincount([k * 3 + l for k, l in keys], minlength=6)
    assert counts.min() > 40                            # roughly uniform (expected 66 each)


def test_coarse_to_fine_schedule_adds_finer_levels_with_progress():
    mp = _mapper("coarse_to_fine", iterations=90)
    levels = [[mp.draw(i)[1] for _ in range(60)] for i in (0, 29, 30, 59, 60, 89)]
    assert set(levels[0]) == {2} and set(levels[1]) == {2}          # first third: coarsest only
    assert set(levels[2]) == {1, 2} and set(levels[3]) == {1, 2}    # then the two coarsest
    assert set(levels[4]) == {0, 1, 2} and set(levels[5]) == {0, 1, 2}


def test_batched_schedule_takes_every_item_at_once_and_bad_names_fail():
    assert _mapper("batched").draw(5) == "all"
    with pytest.raises(ValueError):
        _mapper("bogus")
