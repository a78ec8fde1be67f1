"""Batched scenes on the GPU: every scene of a batched step equals its own single-scene step
bit for bit (the single-scene path is the one checked against the oracle), whatever the
schedule; argument errors are reported before any device work."""
import numpy as np
import pytest

from paper_2512_06230_amd import scenarios as sc

pytestmark = pytest.mark.gpu

FIELDS = ("inst_lab", "inst_m", "inst_P", "inst_src", "hyp_logw", "hyp_off", "hyp_idx", "hyp_parent",
          "birth_lab", "birth_m", "birth_P", "birth_r")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _setup(n, steps, seed=0):
    specs = sc.batch_specs(n, seed=seed, n_min=3, n_max=40, h_lo=16, h_hi=512, n_steps=steps)
    scenes = [sc.make_scene(s, n_steps=steps) for s, _ in specs]
    params = [sc.filter_params(s, h, 1e-5) for s, h in specs]
    return specs, scenes, params


def _concat(torch, scenes, k):
    zs = [sc_.meas[k] for sc_ in scenes]
    off = np.concatenate([[0], np.cumsum([z.shape[0] for z in zs])]).astype(np.int32)
    z = np.concatenate(zs, axis=0) if off[-1] else np.zeros((0, 2), np.float32)
    return torch.as_tensor(np.ascontiguousarray(z, np.float32).reshape(-1, 2), device="cuda"), off


def _run_batch(torch, scenes, params, steps, workers, ljf):
    from paper_2512_06230_amd.glmb import Batch
    b = Batch(params, workers=workers)
    b.set_schedule(workers, ljf)
    for i, s in enumerate(scenes):
        b.scene(i).import_state(sc.warm_start_state(s))
    for k in range(steps):
        z, off = _concat(torch, scenes, k)
        b.step(k, z, off)
    out = [b.scene(i).export_state() for i in range(len(scenes))]
    st = b.stats()
    b.close()
    return out, st


def test_batch_equals_single_scene_steps(torch_cuda):
    from paper_2512_06230_amd.glmb import Tracker
    steps = 3
    specs, scenes, params = _setup(12, steps)
    got, st = _run_batch(torch_cuda, scenes, params, steps, 4, True)
    assert st["n_scenes"] == 12 and st["first_error_scene"] == -1
    for i, (s, p) in enumerate(zip(scenes, params)):
        t = Tracker(p)
        t.import_state(sc.warm_start_state(s))
        for k in range(steps):
            t.predict(k)
            t.update(k, s.meas[k])
            t.truncate(p["h_max"], p["tau"])
        ref = t.export_state()
        t.close()
        for f in FIELDS:
            np.testing.assert_array_equal(got[i][f], ref[f], err_msg="scene %d field %s" % (i, f))


def test_batch_result_does_not_depend_on_the_schedule(torch_cuda):
    steps = 2
    specs, scenes, params = _setup(9, steps, seed=7)
    a, _ = _run_batch(torch_cuda, scenes, params, steps, 1, False)
    b, st = _run_batch(torch_cuda, scenes, params, steps, 8, True)
    assert st["workers"] == 8 and st["longest_first"] == 1
    for x, y in zip(a, b):
        for f in FIELDS:
            np.testing.assert_array_equal(x[f], y[f])


def test_batch_argument_errors(torch_cuda):
    from paper_2512_06230_amd.glmb import Batch, GlmbError
    specs, scenes, params = _setup(3, 1)
    b = Batch(params, workers=2)
    z, off = _concat(torch_cuda, scenes, 0)
    bad = off.copy()
    bad[1], bad[2] = bad[2], bad[1] - 1  # decreasing
    with pytest.raises(GlmbError):
        b.step(0, z, bad)
    with pytest.raises(GlmbError):
        b.set_schedule(0)
    with pytest.raises(GlmbError):
        b.set_schedule(17)
    b.step(0, z, off)  # still usable
    b.close()
