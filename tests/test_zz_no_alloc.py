"""The allocation-free FusedMMA forward (fmm_fusedmm_a_noalloc) against the entry point
it is a variant of (fmm_fusedmm_a with a caller workspace), bit for bit: two calls in a
row, the second on a smaller pattern (the library's scratch array keeps the first call's
partials, which must not leak into the second), with split lines so that the array is
used, in float32 and bfloat16 storage.  Sizes beyond the array are refused."""
import pytest
import torch

import paper_2203_07673_amd as F
from tests.gates import TOL_BF16, TOL_F32
from tests.gpu_helpers import dev, gate, host, log, ref_fusedmm_a
from workloads import dense_normal, rmat

pytestmark = pytest.mark.gpu


def _pattern(scale, seed):
    S = rmat(scale, 16, seed=seed)
    P = F.Pattern.from_csr(S, long_len=64, chunk=32)
    assert P.schedules["csr"] is not None and P.schedules["csr"]["n_chunks"] > 0
    return S, P


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_noalloc_matches_workspace_call_on_two_calls(dtype):
    big, small = _pattern(13, 901), _pattern(10, 902)
    r = 64
    for k, (S, P) in enumerate((big, small)):
        A, B = dense_normal(S.m, r, 910 + k), dense_normal(S.n, r, 920 + k)
        Ad, Bd = dev(A), dev(B)
        if dtype == torch.bfloat16:
            Ad, Bd = F.to_bf16(Ad), F.to_bf16(Bd)
        log(f"noalloc call {k}: m={S.m} nnz={S.nnz} dtype={dtype} chunks={P.schedules['csr']['n_chunks']}")
        want, _ = F.fusedmm_a_raw(P, Ad, Bd)
        got = torch.full_like(want, float("nan"))
        F.fusedmm_a_noalloc_raw(P, Ad, Bd, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {k}: differs from fmm_fusedmm_a"
        ref, mag = ref_fusedmm_a(S, A, B)
        gate(f"noalloc call {k}", host(got), ref, mag, TOL_F32 if dtype == torch.float32 else TOL_BF16)


def test_noalloc_refuses_partials_beyond_its_array():
    S = rmat(15, 16, seed=903)
    P = F.Pattern.from_csr(S, long_len=8, chunk=8)
    r = 1024
    need = P.schedules["csr"]["n_chunks"] * r * 4
    assert need > F.NOALLOC_SCRATCH_BYTES
    log(f"noalloc refusal: partials need {need} bytes")
    A, B = dev(dense_normal(S.m, r, 930)), dev(dense_normal(S.n, r, 931))
    out = torch.zeros(S.m, r, device="cuda")
    with pytest.raises(F.FmmError) as ei:
        F.fusedmm_a_noalloc_raw(P, A, B, out)
    assert ei.value.name == "FMM_ERR_WORKSPACE"
    assert not out.any()
