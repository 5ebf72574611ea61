"""cube2_pp_force_noalloc (the PP force with its scratch in the library's
fixed device array, for callers that cannot allocate) against cube2_pp_force
through the C ABI: bit for bit, on two calls in a row on one context, the
second with a smaller particle set (a prefix of the first's inputs, packed
again), and with accumulate; then once more on a second context of another
mesh size, whose tile order needs a different part of the array."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pp_pair(m, c, x):
    pos, cs, _ = c.pack(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    ref = c.pp_force(pos, cs)
    out = torch.full_like(ref, float("nan"))
    m.cube2_pp_force_noalloc(c.ctx, pos, cs, out)
    torch.cuda.synchronize()
    return pos, cs, ref, out


def test_noalloc_pp_equals_pp_force():
    import paper_2512_12629_amd as m
    x = synthetic.clustered(32, 0.25, 8, 512, 0.5 / 64, 911)
    c = m.Cube2(m.Config(n_fine=64, coarse_ratio=4), n_max=x.shape[1])
    pos, cs, ref, out = _pp_pair(m, c, x)
    assert torch.equal(out, ref)
    # second call, smaller input: the first 10000 particles
    pos2, cs2, ref2, out2 = _pp_pair(m, c, x[:, :10000])
    assert torch.equal(out2, ref2)
    # accumulate adds the same values as the accumulating cube2_pp_force
    base = torch.ones_like(ref2)
    want = c.pp_force(pos2, cs2, base.clone())
    got = base.clone()
    m.cube2_pp_force_noalloc(c.ctx, pos2, cs2, got, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    # another context and mesh size on the same device
    y = synthetic.uniform(20000, 912)
    c3 = m.Cube2(m.Config(n_fine=128), n_max=y.shape[1])
    _, _, ref3, out3 = _pp_pair(m, c3, y)
    assert torch.equal(out3, ref3)
