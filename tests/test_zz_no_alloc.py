"""The allocation-free batched update (sketch_update_batch_noalloc) against
sketch_update_batch through the C ABI: same sketches bit for bit over two
calls in a row, the second with fewer rows; oversized batches rejected with
the state unchanged."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import note

pytestmark = pytest.mark.gpu


def _rows(shapes, base, seed):
    return [torch.from_numpy(synth.lowrank_rows(base + 37 * i, d, np.linspace(3, 0.5, 12), 0.1,
                                                seed=seed + i).astype(np.float32)).cuda()
            for i, (d, ell, _) in enumerate(shapes)]


def test_noalloc_batch_equals_batch_over_two_calls():
    import paper_2601_02019_amd as sk
    shapes = [(64, 8, "exact"), (128, 16, "rand"), (96, 12, "rand"), (300, 136, "rand"), (200, 20, "exact")]
    first = _rows(shapes, 700, 60)      # several shrinks per sketch
    second = _rows(shapes, 90, 80)      # a smaller second call
    mk = lambda i: sk.Sketch(shapes[i][0], shapes[i][1], shrink=shapes[i][2], state_dtype="f32",
                             proj_dtype="bf16", seed=4, stream_id=i)
    ref = [mk(i) for i in range(len(shapes))]
    na = [mk(i) for i in range(len(shapes))]
    note("noalloc: reference batch, two calls")
    sk.sketch_update_batch(ref, first)
    sk.sketch_update_batch(ref, second)
    note("noalloc: allocation-free batch, two calls in a row")
    sk.sketch_update_batch_noalloc(na, first)
    sk.sketch_update_batch_noalloc(na, second)
    for i in range(len(shapes)):
        assert na[i].info()["shrinks"] == ref[i].info()["shrinks"] > 0
        assert torch.equal(na[i].query(), ref[i].query()), i
    for h in ref + na:
        h.close()


def test_noalloc_rejects_batches_beyond_the_scratch():
    import paper_2601_02019_amd as sk
    s = sk.Sketch(8, 2, shrink="exact")
    rows = torch.ones(3 * 9000, 8, dtype=torch.float64, device="cuda")  # > 16384 tasks at ell = 2
    with pytest.raises(sk.SketchError) as e:
        sk.sketch_update_batch_noalloc([s], [rows])
    assert e.value.code == sk.SK_EINVAL
    assert s.info()["rows_seen"] == 0
    sk.sketch_update_batch_noalloc([s], [rows[:30]])
    ref = sk.Sketch(8, 2, shrink="exact")
    ref.update(rows[:30])
    assert torch.equal(s.query(), ref.query())
    s.close()
    ref.close()
