"""The allocation-free RHS entry point (teno_rhs_noalloc) against teno_rhs:
bit-identical RHS, speeds and status on two calls in a row, the second on a
smaller grid (the shared scratch keeps the first call's contents)."""
import numpy as np
import pytest

from paper_2003_09145_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def test_rhs_noalloc_matches_rhs(torch):
    from paper_2003_09145_amd import binding as B
    cases = [
        W.uniform_problem(3, [70, 66, 64], [0.0] * 3, [1.0] * 3,
                          ["periodic", "reflective", "transmissive"]),
        W.uniform_problem(2, [37, 29], [0.0, 0.0], [1.0, 1.0], ["transmissive", "periodic"]),
    ]
    for k, prob in enumerate(cases):
        U = torch.from_numpy(W.random_field(prob, seed=50 + k)).cuda()
        g = B.grid(prob)
        ws = torch.empty(B.workspace_bytes(g), dtype=torch.uint8, device="cuda")
        ref = torch.empty_like(U)
        a_ref = torch.zeros(3, dtype=torch.float64, device="cuda")
        s_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
        B.teno_rhs(g, U, ref, ws, alpha_out=a_ref, status=s_ref)
        out = torch.full_like(U, np.nan)
        a_out = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
        s_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        B.teno_rhs_noalloc(g, U, out, alpha_out=a_out, status=s_out)
        # frozen speeds through the same scratch
        out2 = torch.full_like(U, np.nan)
        B.teno_rhs_noalloc(g, U, out2, alpha_in=a_ref)
        torch.cuda.synchronize()
        print(f"[no-alloc] {prob.n}: bitwise {bool(torch.equal(out, ref))}", flush=True)
        assert torch.equal(out, ref) and torch.equal(out2, ref)
        assert torch.equal(a_out, a_ref) and torch.equal(s_out, s_ref)
