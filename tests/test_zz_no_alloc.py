"""vmc_step_noalloc (the step for callers that cannot allocate: its
workspace is a fixed device array of the library) against vmc_step with a
caller workspace, through the C ABI: two calls in a row, the second on a
smaller input, each equal to vmc_step bit for bit; an input whose workspace
exceeds the fixed array is refused before any launch."""
import numpy as np
import pytest

from paper_2507_18700_amd import synth
from tests.gpu_util import lib_and_oracle, torch_gpu

pytestmark = pytest.mark.gpu


def _outs(torch, V, gm, ns):
    return (torch.empty((ns, gm.N), dtype=torch.uint8, device="cuda"),
            torch.empty(ns, dtype=torch.float32, device="cuda"),
            torch.empty(ns, dtype=torch.float32, device="cuda"),
            torch.empty((ns, 2), dtype=torch.float64, device="cuda"),
            torch.empty(V.param_count(gm), dtype=torch.float64, device="cuda"),
            torch.empty(4, dtype=torch.float64, device="cuda"))


def test_noalloc_step_equals_vmc_step():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    assert V.noalloc_scratch_bytes() == 256 << 20
    calls = [
        # (dims, Lx, Ly, d_h, complex, glu, bf16, Hamiltonian, ns): the second is smaller
        (2, 5, 4, 32, True, True, True, V.ham(V.VMC_HEISENBERG, 1.0, 0.0, True), 300),
        (1, 12, 1, 16, False, False, False, V.ham(V.VMC_TFIM, 1.0, 1.0), 77),
    ]
    for i, (dims, Lx, Ly, dh, cplx, glu, bf16, H, ns) in enumerate(calls):
        spec, gm, _ = lib_and_oracle(dims, Lx, Ly, dh, cplx, glu, bf16)
        p = torch.from_numpy(synth.xavier_params(spec, 40 + i, bias_scale=0.2)).cuda()
        ref = V.vmc_step(gm, p, H, ns, seed=3, counter=i, out=_outs(torch, V, gm, ns))
        got = V.vmc_step_noalloc(gm, p, H, ns, _outs(torch, V, gm, ns), seed=3, counter=i)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), "call %d" % i
        st = got[5].cpu().numpy()
        assert np.isfinite(st).all() and st[3] == 0


def test_noalloc_refuses_inputs_above_the_fixed_workspace():
    torch = torch_gpu()
    from paper_2507_18700_amd import vmcrnn as V
    spec, gm, _ = lib_and_oracle(2, 10, 10, 128, False, True, True)
    H = V.ham(V.VMC_TFIM, 1.0, 3.0)
    ns = 10000
    assert V.workspace_size(gm, H, ns) > V.noalloc_scratch_bytes()
    p = torch.from_numpy(synth.xavier_params(spec, 1)).cuda()
    out = _outs(torch, V, gm, ns)
    with pytest.raises(V.VmcError) as ei:
        V.vmc_step_noalloc(gm, p, H, ns, out)
    assert ei.value.status == V.VMC_ENOSPACE
