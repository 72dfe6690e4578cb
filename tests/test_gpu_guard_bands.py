"""Guard bands: every output buffer and every workspace sits inside a larger
allocation whose margins hold a sentinel byte pattern; each entry point runs
once at ragged shapes (image sides 160, 192, 320, 384; slice and coil counts
that are not multiples of any block size), and the margins must come back
untouched.  Inputs are checked unchanged too.  This catches stores past the end
(or before the start) of a buffer that a norm-wise parity check would not see.
"""

import numpy as np
import pytest

from tests.gpu_util import c64, random_case, to_dev

pytestmark = pytest.mark.gpu

GUARD = 4096          # bytes of sentinel on each side (keeps 256-byte alignment)
SENTINEL = 0xA5


class Guarded:
    def __init__(self, shape, dtype):
        import torch
        self.numel = int(np.prod(shape))
        self.nbytes = self.numel * torch.empty((), dtype=dtype).element_size()
        self.buf = torch.full((GUARD + self.nbytes + GUARD,), SENTINEL, dtype=torch.uint8, device="cuda")
        self.t = self.buf[GUARD:GUARD + self.nbytes].view(dtype).view(shape)

    def intact(self):
        import torch
        torch.cuda.synchronize()
        return bool((self.buf[:GUARD] == SENTINEL).all()) and bool((self.buf[GUARD + self.nbytes:] == SENTINEL).all())


def guarded_like(a):
    import torch
    g = Guarded(a.shape, a.dtype)
    g.t.copy_(a)
    return g


CASES = [(160, 5, 3, 4, 0), (192, 7, 2, 3, 0), (320, 3, 3, 4, 0), (384, 5, 3, 4, 1), (160, 3, 2, 4, 2)]


@pytest.mark.parametrize("n,coils,slices,levels,kind", CASES)
def test_entry_points_write_only_their_outputs(n, coils, slices, levels, kind):
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, w = random_case(n, coils, slices, "1d" if kind == 1 else "2d", seed=n + coils)
    plan = pf.Plan(n, coils, slices, haar_levels=levels, mask_kind=kind)
    ws = Guarded(tuple(plan.ws.shape), torch.uint8)
    plan.ws = ws.t
    inputs = {"sens": to_dev(sens), "x": to_dev(x), "w": to_dev(w)}
    if kind == pf.TOEPLITZ:
        rng = np.random.default_rng(n)
        inputs["mask"] = to_dev(rng.random((slices, 2 * n, 2 * n)).astype(np.float32))
    else:
        inputs["mask"] = to_dev(mask)
    gin = {k: guarded_like(v) for k, v in inputs.items()}
    before = {k: v.t.clone() for k, v in gin.items()}
    ts, tm, tx, tw = (gin[k].t for k in ("sens", "mask", "x", "w"))
    img = (slices, n, n)
    outs = []

    def out(shape, dtype=torch.complex64):
        g = Guarded(shape, dtype)
        outs.append(g)
        return g.t

    pf.normal_apply(plan, ts, tm, tx, out(img), 0.5, w=tw, beta=0.25)
    pf.poly_apply(plan, ts, tm, 0.9, [4.0, -10.0 / 3.0], tx, out(img))
    if kind == pf.MASK_1D:
        packed = pf.pack_coil_maps(plan, ts, out((plan.n_coil,)))
        pf.normal_apply_packed(plan, packed, tm, tx, out(img), 0.5, w=tw, beta=0.25)
        pf.poly_apply_packed(plan, packed, tm, 0.9, [4.0, -10.0 / 3.0], tx, out(img))
    xn, zn, red = out(img), out(img), out((3,), torch.float64)
    pf.step(plan, tx, tw, tw, xn, zn, 0.05, 0.25, red)
    if kind != pf.TOEPLITZ:
        k = out((slices, coils, n, n))
        pf.forward(plan, ts, tm, tx, k)
        pf.adjoint(plan, ts, tm, k, out(img), 1.0)
        pf.data_term(plan, ts, tm, k, tx, 1.0, 0.5)
        b = k
        bnorm = 0.0
    else:
        b = tx
        bnorm = 3.0
    v = out(img)
    v.copy_(tx)
    pf.power_iteration(plan, ts, tm, 3, v=v)
    xs, zs = out(img), out(img)
    # 4 iterations of d = 2 (12 applies): a phase-encode solve packs its coil maps into the workspace
    pf.solve(plan, ts, tm, b, xs, 1e-3, degree=2, max_iter=4, inv_l=0.5, z=zs, check_every=2,
             eval_objective=True, bnorm=bnorm)
    torch.cuda.synchronize()
    assert ws.intact(), "workspace margins written"
    for i, g in enumerate(outs):
        assert g.intact(), f"output {i} margins written"
    for key, g in gin.items():
        assert g.intact(), f"input {key} margins written"
        assert torch.equal(g.t, before[key]), f"input {key} changed"


@pytest.mark.parametrize("n,coils,slices,levels", [(192, 5, 3, 3), (160, 7, 2, 4)])
def test_unrolled_and_batch_write_only_their_outputs(n, coils, slices, levels):
    import torch
    import paper_2204_10252_amd as pf
    sens, mask, x, w = random_case(n, coils, slices, "2d", seed=7 * n)
    plan = pf.Plan(n, coils, slices, haar_levels=levels)
    ts, tm = to_dev(sens), to_dev(mask)
    k = torch.empty((slices, coils, n, n), dtype=torch.complex64, device="cuda")
    pf.forward(plan, ts, tm, to_dev(x), k)
    u = pf.Unrolled(plan, 2, 5, 0.5, ckpt_every=2)
    uws = Guarded(tuple(u.ws.shape), torch.uint8)
    u.ws = uws.t
    ck = Guarded(tuple(u.ckpt.shape), torch.uint8)
    xo = Guarded((slices, n, n), torch.complex64)
    coef = [4.0, -10.0 / 3.0, 0.5]
    u.forward(ts, tm, k, xo.t, 1e-3, coef, ckpt=ck.t)
    u.backward(ts, tm, to_dev(w), 1e-3, coef, ckpt=ck.t)
    for name, g in (("workspace", uws), ("checkpoints", ck), ("x", xo)):
        assert g.intact(), f"unrolled {name} margins written"
    # a batch of uneven slices (sides 160 and 192, odd coil counts)
    shapes = [(160, 3, 4), (192, 5, 3), (160, 1, 2)]
    batch = pf.Batch(shapes)
    bws = Guarded(tuple(batch.ws.shape), torch.uint8)
    batch.ws = bws.t
    sl_sens, sl_mask, sl_b, sl_x = [], [], [], []
    for i, (nn, cc, _) in enumerate(shapes):
        s_, m_, x_, _ = random_case(nn, cc, 1, "2d", seed=100 + i)
        pl = pf.Plan(nn, cc, 1, haar_levels=2)
        bb = torch.empty((cc, nn, nn), dtype=torch.complex64, device="cuda")
        pf.forward(pl, to_dev(s_[0]), to_dev(m_[0]), to_dev(x_[0]), bb)
        sl_sens.append(to_dev(s_[0]))
        sl_mask.append(to_dev(m_[0]))
        sl_b.append(bb)
        sl_x.append(Guarded((nn, nn), torch.complex64))
    pf.batch_solve(batch, sl_sens, sl_mask, sl_b, [g.t for g in sl_x], [1e-3] * 3, degree=2, max_iter=3,
                   inv_l=[0.5] * 3, eval_objective=True, check_every=3)
    assert bws.intact(), "batch workspace margins written"
    for i, g in enumerate(sl_x):
        assert g.intact(), f"batch slice {i} margins written"
