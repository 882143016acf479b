"""GPU parity of ifsvgp_adam against the float64 Adam oracle (oracle/optim.py).

Several consecutive steps with changing gradients, on a ragged size and on a
parameter block of Z's shape.  The kernel computes in fp32 from fp32 state, so
each step carries fp32 rounding of its few operations.  That rounding is
relative to the operands (beta1 |m| + (1 - beta1) |g| for the first moment),
not to the result, which can be small where the two terms cancel: the gate is
relative 2e-6 plus an absolute 1e-6 of the array's largest magnitude (a few
ulps of the operand scale after six steps)."""
import numpy as np
import pytest

from oracle import optim

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape,ascend", [((1001,), False), ((1024, 16), True), ((1,), False)])
def test_adam_parity(shape, ascend):
    from paper_2604_00697_amd.lib import Context
    dev = torch.device("cuda", 0)
    g = np.random.Generator(np.random.PCG64(sum(shape)))
    ctx = Context(8, 8, 2, "fp32")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    p0 = g.standard_normal(shape).astype(np.float32)
    P, Mo, Vo = f32(p0), f32(np.zeros(shape)), f32(np.zeros(shape))
    p, m, v = p0.astype(np.float64), np.zeros(shape), np.zeros(shape)
    for t in range(1, 7):
        gr = (g.standard_normal(shape) * 10.0 ** g.uniform(-3, 1)).astype(np.float32)
        ctx.adam(P, f32(gr), Mo, Vo, t, lr=2e-2, beta1=0.85, beta2=0.99, eps=1e-7, ascend=ascend)
        p, m, v = optim.adam_step(p, gr, m, v, t, lr=2e-2, beta1=0.85, beta2=0.99, eps=1e-7,
                                  ascend=ascend)
        torch.cuda.synchronize()
        print(f"ADAM shape={shape} ascend={ascend} step={t}", flush=True)
        for name, a, r in (("param", P, p), ("m", Mo, m), ("v", Vo, v)):
            np.testing.assert_allclose(a.cpu().numpy(), r, rtol=2e-6,
                                       atol=1e-6 * float(np.max(np.abs(r))), err_msg=name)
    assert ctx.status() == 0
    ctx.close()


def test_adam_argument_errors():
    from paper_2604_00697_amd.lib import Context, IFSVGPError
    dev = torch.device("cuda", 0)
    ctx = Context(8, 8, 2, "fp32")
    x = torch.zeros(4, device=dev)
    with pytest.raises(IFSVGPError):
        ctx.adam(x, x, x, x, 0)            # step must be >= 1
    with pytest.raises(IFSVGPError):
        ctx.adam(x, x, x, x, 1, beta1=1.0)  # decay must be < 1
    ctx.close()
