"""tina_pfb_execute_noalloc: the allocation-free execute (static device
scratch instead of the plan's workspace) gives the same output as
tina_pfb_execute, bit for bit (the same kernels run), on two calls in a row
with the second smaller, with and without a state; sizes beyond the scratch
are refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _x(n, seed, cplx=False):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal(n)
    if cplx:
        x = x + 1j * g.standard_normal(n)
        return x.astype(np.complex64)
    return x.astype(np.float32)


def _bits(t):
    t = t.cpu()
    return torch.view_as_real(t).numpy() if t.is_complex() else t.numpy()


CASES = [  # (P, M, sample type, precision (/DFT algorithm), output, samples of the first call)
    (1024, 16, "r32", "fp32", "pfb", 1024 * 3000 + 517),
    (1024, 12, "r32", "fp8", "pfb", 1024 * 2500 + 3),
    (512, 16, "c64", "bf16x3", "pfb", 512 * 2049 + 100),
    (256, 8, "c64", "fp16x3", "pfb", 256 * 3000 + 9),
    (1024, 16, "r32", "mxfp8", "pfb", 1024 * 1500),
    (4096, 8, "c64", "fp32", "fir", 4096 * 700 + 5),
    (4096, 8, "c64", "fp32/factored", "pfb", 4096 * 600 + 7),
    (1024, 16, "r32", "fp32/table", "pfb", 1024 * 900 + 33),
]


@pytest.mark.parametrize("P,M,st,prec,out,n1", CASES)
def test_noalloc_equals_execute_two_calls(P, M, st, prec, out, n1):
    from paper_2408_16551_amd.pfb import Plan
    print(f"noalloc: P={P} M={M} {st} {prec} {out} n1={n1}", flush=True)
    cplx = st == "c64"
    form, dft = (prec.split("/") + ["dense"])[:2]
    plan = Plan(P, M, st, "hann", form, out, dft=dft)
    for n, seed in ((n1, 1), (n1 // 3 + 11, 2)):  # the second call is smaller
        x = torch.from_numpy(_x(n, seed, cplx)).cuda()
        ref = plan(x).clone()
        got = torch.full_like(ref, float("nan"))
        plan.execute(x, out=got, noalloc=True)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(got), _bits(ref)), (n, prec)
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
def test_noalloc_streaming_without_a_plan_workspace(prec):
    """A plan made without a workspace runs only through the allocation-free
    call; chunks with a state equal the workspace plan's chunks bit for bit."""
    from paper_2408_16551_amd.pfb import Plan, State, TinaError
    P, M = 1024, 16
    print(f"noalloc streaming: P={P} M={M} {prec}", flush=True)
    ref_plan = Plan(P, M, "r32", "hann", prec)
    bare = Plan(P, M, "r32", "hann", prec, workspace_bytes=-1)
    x = torch.from_numpy(_x(P * 5000 + 300, 7)).cuda()
    with pytest.raises(TinaError):
        bare(x)  # no workspace: tina_pfb_execute refuses
    s_ref, s_bare = State(ref_plan), State(bare)
    cuts = [0, 777, P * 2000 + 5, P * 2001, x.numel()]
    for a, b in zip(cuts[:-1], cuts[1:]):
        r = ref_plan(x[a:b], state=s_ref).clone()
        g = torch.full_like(r, float("nan"))
        g = bare.execute(x[a:b], out=g, state=s_bare, noalloc=True)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(g), _bits(r)), (a, b)
    for o in (s_ref, s_bare, ref_plan, bare):
        o.close()


def test_noalloc_refuses_more_frames_than_the_scratch_holds():
    """Through the C ABI directly: 64 MiB hold 16384 frames of P = 1024 real
    FP32; 16385 frames return TOO_LARGE and leave the output untouched."""
    from paper_2408_16551_amd.pfb import Plan, load
    lib = load()
    P = 1024
    plan = Plan(P, 4, "r32", "hann", "fp32", workspace_bytes=-1)
    for frames, want in ((16384, 0), (16385, 7)):
        x = torch.zeros(frames * P, dtype=torch.float32, device="cuda")
        out = torch.full((frames, P // 2 + 1), 3.0, dtype=torch.complex64, device="cuda")
        fw = ctypes.c_int64(-1)
        st = lib.tina_pfb_execute_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), frames * P,
                                          ctypes.c_void_p(out.data_ptr()), frames, None, ctypes.byref(fw),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert st == want, lib.tina_last_error()
        if want == 0:
            assert fw.value == frames and bool((out == 0).all())
        else:
            assert b"static scratch" in lib.tina_last_error() and bool((out == 3.0).all())
    plan.close()
