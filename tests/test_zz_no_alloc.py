"""kernel_matvec_noalloc (scratch in a static device array, no allocation by
the library) against kernel_matvec_ex on the same inputs: the two run the
same kernels on the same scratch layout, so the outputs agree bit for bit.
Calls follow each other with shrinking inputs, so a later call runs on the
array as the earlier one left it."""
import numpy as np
import pytest

from paper_2304_05460_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def afn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05460_amd import afn as mod
    mod.lib()
    return mod


def _colmajor(A):
    return torch.tensor(np.ascontiguousarray(A.T), dtype=torch.float64, device="cuda").t()


# (n, d, l, nrhs, precision, kernel): pruned tile path, FP32, many columns,
# the plain path above d = 8 and below the pruning size, Matern-3/2
CASES = [(60000, 3, 0.05, 1, 0, 0), (20000, 3, 0.1, 1, 1, 0), (6000, 3, 0.1, 7, 0, 0),
         (9000, 8, 2.0, 1, 0, 0), (5000, 12, 3.0, 2, 1, 0), (3000, 3, 0.2, 1, 0, 1)]


def test_noalloc_equals_kernel_matvec_on_shrinking_calls(afn):
    for n, d, l, nrhs, prec, kind in CASES:
        print(f"noalloc n={n} d={d} nrhs={nrhs} prec={prec} kernel={kind}", flush=True)
        X = torch.tensor(W.points("uniform" if d == 3 else "normal", n, d, 91), device="cuda")
        V = np.random.default_rng(92).standard_normal((n, nrhs))
        v = _colmajor(V) if nrhs > 1 else torch.tensor(V[:, 0], device="cuda")
        ref = afn.kernel_matvec(X, l, 1e-3, v, precision=prec, kernel=kind)
        out = torch.full_like(ref, float("nan"))
        afn.kernel_matvec_noalloc(X, l, 1e-3, v, out, precision=prec, kernel=kind)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
        # a second call on the same inputs after the array was reused
        out2 = torch.full_like(ref, float("nan"))
        afn.kernel_matvec_noalloc(X, l, 1e-3, v, out2, precision=prec, kernel=kind)
        assert torch.equal(out2, ref)


def test_noalloc_rejects_inputs_beyond_the_static_area(afn):
    n = 400000
    X = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(v)
    with pytest.raises(afn.AFNError) as e:
        afn.kernel_matvec_noalloc(X, 0.1, 1e-3, v, out)
    assert e.value.status == afn.AFN_EINVAL
    assert "static area" in str(e.value)
