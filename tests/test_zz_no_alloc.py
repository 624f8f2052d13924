"""dd_forward_noalloc (the forward on the library's static workspace, for
callers that cannot allocate) against dd_forward: two calls in a row, the
second with a smaller input, on uint8 (bit-exact) and float32 plans (same
kernels, so bit-identical too), plus its error paths."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
dd = pytest.importorskip("paper_1912_07704_amd")
from paper_1912_07704_amd import _lib  # noqa: E402

DD_ERR_INVALID, DD_ERR_WORKSPACE = -2, -9
WS_MAX = 64 << 20


def say(*a):
    print("[case]", *a, flush=True)


def call_noalloc(plan, x, out, w=None):
    """The C ABI call itself (ctypes), on torch's current stream."""
    L = _lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.dd_forward_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                None if w is None else ctypes.c_void_p(w.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), out.numel(), s)


CASES = [
    # (dtype, nchans, nsamp, ranges): the second of each pair is smaller
    ("u8", 256, 40000, [(0.0, 60.0, 0.5, 1), (60.0, 120.0, 1.0, 2), (120.0, 200.0, 2.0, 4)]),
    ("u8", 96, 9000, [(0.0, 30.0, 1.0, 1), (30.0, 50.0, 2.0, 3)]),
    ("f32", 128, 30000, [(0.0, 40.0, 1.0, 1), (40.0, 80.0, 2.0, 2)]),
    ("f32", 33, 5000, [(0.0, 20.0, 1.0, 1)]),
]


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_noalloc_equals_forward_twice(dtype):
    cases = [c for c in CASES if c[0] == dtype]
    rng = np.random.default_rng(4242)
    for i, (_, nch, nsamp, ranges) in enumerate(cases):
        freqs = synth.band_freqs(1500.0, 1250.0, nch)
        tsamp = 2.56e-4
        plan = dd.Plan(freqs, tsamp, nsamp, ranges, dtype)
        say("noalloc", dtype, i, nch, nsamp, ranges, plan.workspace_bytes)
        plan.prepare()
        if dtype == "u8":
            x = torch.from_numpy(rng.integers(0, 256, (nch, nsamp)).astype(np.uint8)).cuda()
            w = None
            odt = torch.int32
        else:
            x = torch.from_numpy(rng.standard_normal((nch, nsamp)).astype(np.float32)).cuda()
            w = torch.from_numpy(rng.uniform(0.5, 1.5, nch).astype(np.float32)).cuda()
            odt = torch.float32
        want = dd.dedisperse(x, plan, weights=w)
        got = torch.full((plan.out_elems + 16,), -7, dtype=odt, device="cuda")
        assert call_noalloc(plan, x, got, w) == 0, _lib.lib().dd_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got[: plan.out_elems], want), f"call {i}"
        assert (got[plan.out_elems:] == -7).all(), "wrote past out_elems"


def test_noalloc_binding_and_errors():
    freqs = synth.band_freqs(1500.0, 1250.0, 64)
    plan = dd.Plan(freqs, 2.56e-4, 6000, [(0.0, 20.0, 1.0, 1)], "u8")
    x = torch.randint(0, 256, (64, 6000), dtype=torch.uint8, device="cuda")
    out = torch.empty(plan.out_elems, dtype=torch.int32, device="cuda")
    # tables not yet on the device: rejected, nothing uploaded or allocated
    assert call_noalloc(plan, x, out) == DD_ERR_INVALID
    plan.prepare()
    dd.dedisperse_noalloc(x, plan, out)
    torch.cuda.synchronize()
    assert torch.equal(out, dd.dedisperse(x, plan))
    # a plan whose binned copies exceed the static workspace
    big = dd.Plan(synth.band_freqs(1500.0, 1250.0, 1024), 2.56e-4, 40000,
                  [(0.0, 10.0, 1.0, 1)], "u8")
    assert big.workspace_bytes > WS_MAX
    big.prepare()
    xb = torch.zeros((1024, 40000), dtype=torch.uint8, device="cuda")
    ob = torch.empty(big.out_elems, dtype=torch.int32, device="cuda")
    assert call_noalloc(big, xb, ob) == DD_ERR_WORKSPACE
    with pytest.raises(dd.DDError):
        dd.dedisperse_noalloc(xb, big, ob)
