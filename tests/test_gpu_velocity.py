"""GPU parity of the IOS velocity codec (section 2.3, linear reading; see
oracle.vel_encode) against the oracle through the C ABI: the bulk velocity
field, the global step and every int16 code bit-exact (both sides take the
integer decisions in the same FP32 arithmetic), the decoded velocities
bit-exact, on seeded inputs with one and two PM levels (bulk cells of 2, 4
and 8 fine cells), a ragged particle count and an empty input."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "uniform_64_one_level": (64, 0, 2, lambda: synthetic.uniform(32 ** 3, 701)),
    "clustered_64_ratio4": (64, 4, 2, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 702)),
    "zel_32_ratio2_ragged": (32, 2, 1, lambda: synthetic.zeldovich(13, 0.25, 703)),
    "clustered_64_ratio8": (64, 8, 3, lambda: synthetic.clustered(20, 0.25, 4, 256, 0.5 / 64, 704)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_velocity_codec_bit_exact(name):
    import paper_2512_12629_amd as m
    n_f, cr, shift, gen = CASES[name]
    x = gen()
    c = m.Cube2(m.Config(n_fine=n_f, coarse_ratio=cr), n_max=x.shape[1])
    assert m.cube2_vel_bulk_side(c.ctx) == n_f >> shift
    pos, cs, _ = c.pack(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    q = oracle.quantize(x, n_f)
    perm, _, _ = oracle.ios_order(q, n_f)
    qs = q[:, perm]
    rng = np.random.default_rng(705 + list(CASES).index(name))
    v = (rng.standard_normal(qs.shape) * 2.5 + 0.75).astype(np.float32)
    vq, vb, sc = c.vel_encode(pos, cs, torch.from_numpy(v).cuda())
    vq_or, vb_or, s_or = oracle.vel_encode(qs, v, n_f, shift)
    assert np.float32(sc.item()) == s_or
    assert np.array_equal(vb.cpu().numpy(), vb_or)
    assert np.array_equal(vq.cpu().numpy(), vq_or)
    back = c.vel_decode(pos, cs, vq, vb, sc).cpu().numpy()
    assert np.array_equal(back, oracle.vel_decode(qs, vq_or, vb_or, s_or, n_f, shift))
    assert c.status() == 0


def test_velocity_codec_empty_input():
    import paper_2512_12629_amd as m
    c = m.Cube2(m.Config(n_fine=32, coarse_ratio=4), n_max=1)
    pos, cs, _ = c.pack(torch.empty((3, 0), dtype=torch.float32, device="cuda"))
    vq, vb, sc = c.vel_encode(pos, cs, torch.empty((3, 0), dtype=torch.float32, device="cuda"))
    assert vq.shape == (3, 0)
    assert float(sc.item()) == 1.0
    assert torch.count_nonzero(vb).item() == 0
