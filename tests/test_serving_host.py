"""Host-side checks of the serving loop's plan pool (no GPU work)."""
import numpy as np

from paper_2010_13213_amd import inputs, serve


def _req(blocks, nb=8, dx0=1.0, nc=1, precision="fp64", levels=None):
    lv = [inputs.Level(blocks=np.asarray(b, dtype=np.int32), values=np.zeros((nc, len(b), nb, nb, nb)))
          for b in (levels or [blocks])]
    return inputs.Request(rid=0, problem=inputs.Problem(nb=nb, dx0=dx0, levels=lv), precision=precision,
                          arrival=0.0)


def test_plan_pool_key_separates_supports_with_equal_block_counts():
    slab = [(x, y, 0) for y in range(4) for x in range(2)]      # 2 x 4 x 1 blocks
    row = [(x, 0, 0) for x in range(8)]                          # 8 x 1 x 1 blocks
    moved = [(x + 1, y, 0) for x, y, _ in slab]                  # same shape, other origin
    keys = {serve.PlanPool.key(_req(b)) for b in (slab, row, moved)}
    assert len(keys) == 3
    assert serve.PlanPool.key(_req(slab)) == serve.PlanPool.key(_req(list(slab)))


def test_plan_pool_key_separates_every_plan_field():
    b = [(0, 0, 0), (1, 0, 0)]
    base = serve.PlanPool.key(_req(b))
    assert serve.PlanPool.key(_req(b, dx0=0.5)) != base
    assert serve.PlanPool.key(_req(b, nc=3)) != base
    assert serve.PlanPool.key(_req(b, precision="fp32_refine")) != base
    assert serve.PlanPool.key(_req(b, nb=16)) != base
    two = serve.PlanPool.key(_req(None, levels=[b, [(0, 0, 0)]]))
    assert two != base
    # the level split matters, not only the concatenated block list
    assert serve.PlanPool.key(_req(None, levels=[b[:1], b[1:]])) != serve.PlanPool.key(_req(b))
