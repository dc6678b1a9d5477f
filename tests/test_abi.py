"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, reports parameter counts that match the documented layout,
and rejects bad arguments before touching any device pointer."""
import ctypes
import os
import re

import pytest

from paper_2507_18700_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vmcrnn.h")
LIB = os.path.join(ROOT, "paper_2507_18700_amd", "libvmcrnn.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:vmc_status|int64_t|size_t|char)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libvmcrnn.so is not built; run __graft_entry__.build()")
    from paper_2507_18700_amd import vmcrnn as V
    return V


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert set(names) == {"vmc_param_count", "vmc_workspace_size", "rnn_sample", "rnn_logpsi", "rnn_logpsi_grad",
                          "local_energy", "vmc_grad", "vmc_energy_stats", "vmc_grad_chunk", "vmc_step", "vmc_step_batched", "vmc_batched_workspace_size",
                          "vmc_step_noalloc", "vmc_noalloc_scratch_bytes",
                          "vmc_adam", "vmc_check_finite", "grow_hidden",
                          "vmc_row_tile_options", "vmc_set_tuning", "vmc_get_tuning", "vmc_autotune_step",
                          "vmc_chain_timing", "vmc_chain_time", "vmc_status_str"}
    L = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(L, n), n
    assert set(lib.EXPORTS) == set(names)


@pytest.mark.parametrize("dims,Lx,Ly,dh,cplx,glu", [(1, 20, 1, 16, 0, 0), (1, 7, 1, 5, 1, 1), (2, 10, 10, 128, 0, 1),
                                                    (2, 3, 5, 20, 1, 0), (2, 16, 16, 256, 1, 1)])
def test_param_count_matches_layout(lib, dims, Lx, Ly, dh, cplx, glu):
    m = lib.model(dims=dims, Lx=Lx, Ly=Ly, d_h=dh, is_complex=cplx, glu=glu)
    spec = synth.ModelSpec(dims=dims, Lx=Lx, Ly=Ly, d_h=dh, is_complex=bool(cplx), glu=bool(glu))
    assert lib.param_count(m) == synth.param_count(spec)


def test_c3_parameter_count(lib):
    # 2D GRU d_h = 128 with GLU: W, W_g [128 x 260], b, b_g, U [128 x 256], GLU, head
    m = lib.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True)
    assert lib.param_count(m) == 2 * 128 * 260 + 2 * 128 + 128 * 256 + 2 * (128 * 128 + 128) + 2 * 128 + 2


def test_invalid_descriptors(lib):
    L = lib.lib()
    bad = [lib.Model(3, 4, 1, 8, 0, 0, 0), lib.Model(1, 4, 2, 8, 0, 0, 0), lib.Model(1, 1, 1, 8, 0, 0, 0),
           lib.Model(1, 8, 1, 0, 0, 0, 0), lib.Model(1, 8, 1, 8, 2, 0, 0), lib.Model(1, 8, 1, 8, 0, 0, 7)]
    for m in bad:
        assert L.vmc_param_count(ctypes.byref(m)) == -1
        out = ctypes.c_size_t(0)
        assert L.vmc_workspace_size(ctypes.byref(m), None, 10, ctypes.byref(out)) == -1
    m = lib.model(dims=1, Lx=8, d_h=300)
    out = ctypes.c_size_t(0)
    assert L.vmc_workspace_size(ctypes.byref(m), None, 10, ctypes.byref(out)) == -2  # d_h > 256


def test_argument_errors_before_launch(lib):
    """Null pointers, a bad Hamiltonian, a small or misaligned workspace:
    rejected on the host; the fake device pointers are never dereferenced."""
    L = lib.lib()
    m = lib.model(dims=2, Lx=4, Ly=4, d_h=16, glu=True)
    H = lib.ham(lib.VMC_TFIM, 1.0, 3.0)
    need = lib.workspace_size(m, H, 100)
    assert need > 0
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    # workspace too small
    assert L.local_energy(ctypes.byref(m), fake, ctypes.byref(H), 100, fake, fake, ws, need - 1, None) == -3
    # misaligned workspace
    assert L.rnn_logpsi(ctypes.byref(m), fake, 100, fake, fake, None, ctypes.c_void_p(0x200004), need, None) == -1
    # null outputs / inputs
    assert L.rnn_sample(ctypes.byref(m), fake, 100, 0, 0, None, None, fake, None, ws, need, None) == -1
    assert L.rnn_logpsi(ctypes.byref(m), None, 100, fake, fake, None, ws, need, None) == -1
    assert L.vmc_grad(ctypes.byref(m), fake, 100, fake, None, None, fake, None, ws, need, None) == -1
    assert L.rnn_logpsi_grad(ctypes.byref(m), fake, 100, fake, None, None, fake, ws, need, None) == -1
    # chunked gradient: the whole set's weights and statistics are required; no samples
    assert L.vmc_grad_chunk(ctypes.byref(m), fake, 100, fake, fake, None, fake, fake, ws, need, None) == -1
    assert L.vmc_grad_chunk(ctypes.byref(m), fake, 100, fake, fake, fake, None, fake, ws, need, None) == -1
    assert L.vmc_grad_chunk(ctypes.byref(m), fake, 100, fake, fake, fake, fake, fake, ws, need - 1, None) == -3
    assert L.vmc_energy_stats(0, fake, None, fake, None) == -1
    assert L.vmc_energy_stats(100, None, None, fake, None) == -1
    assert L.vmc_energy_stats(100, fake, None, None, None) == -1
    assert L.rnn_logpsi_grad(ctypes.byref(m), fake, 100, fake, fake, None, fake, ws, need - 1, None) == -3
    assert L.local_energy(ctypes.byref(m), fake, None, 100, fake, fake, ws, need, None) == -1
    badH = lib.Ham(5, 0, 1.0, 1.0)
    assert L.local_energy(ctypes.byref(m), fake, ctypes.byref(badH), 100, fake, fake, ws, need, None) == -1
    assert L.rnn_logpsi(ctypes.byref(m), fake, 0, fake, fake, None, ws, need, None) == -1
    # grow_hidden: shrinking, negative noise, partial moment sets
    assert L.grow_hidden(ctypes.byref(m), fake, 8, 0, 0.0, fake, None, None, None, None, None) == -1
    assert L.grow_hidden(ctypes.byref(m), fake, 32, 0, -1.0, fake, None, None, None, None, None) == -1
    assert L.grow_hidden(ctypes.byref(m), fake, 32, 0, 0.0, fake, fake, None, None, None, None) == -1
    # autotuner: repetition count, workspace and outputs checked before any event or launch
    t = lib.Tuning()
    args = (ctypes.byref(m), fake, ctypes.byref(H), 100, 0, 0, None, fake, fake, None, fake, fake, fake)
    assert L.vmc_autotune_step(*args, ws, need, None, 0, ctypes.byref(t)) == -1
    assert L.vmc_autotune_step(*args, ws, need, None, 101, ctypes.byref(t)) == -1
    assert L.vmc_autotune_step(*args, ws, need - 1, None, 3, ctypes.byref(t)) == -3
    assert L.vmc_autotune_step(ctypes.byref(m), fake, ctypes.byref(H), 100, 0, 0, None, None, fake, None, fake,
                               fake, fake, ws, need, None, 3, ctypes.byref(t)) == -1
    assert L.vmc_status_str(-3) == b"workspace too small"


def test_nonfinite_and_hamiltonian_errors(lib):
    """Non-finite couplings, noise and Adam settings give VMC_ENONFINITE, the
    1D-only Hamiltonians on a 2D lattice VMC_EUNSUPPORTED, all on the host
    before any launch (the fake device pointers are never dereferenced)."""
    L = lib.lib()
    inf, nan = float("inf"), float("nan")
    m1 = lib.model(dims=1, Lx=12, d_h=16)
    m2 = lib.model(dims=2, Lx=4, Ly=4, d_h=16, glu=True)
    out = ctypes.c_size_t(0)
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    for H in (lib.ham(lib.VMC_TFIM, nan, 1.0), lib.ham(lib.VMC_TFIM, 1.0, inf),
              lib.ham(lib.VMC_LRTFIM, 1.0, 1.0, alpha=nan), lib.ham(lib.VMC_CLUSTER, -inf, 0.0),
              lib.ham(lib.VMC_HEISENBERG, nan, 0.0, True)):
        assert L.vmc_workspace_size(ctypes.byref(m1), ctypes.byref(H), 10, ctypes.byref(out)) == lib.VMC_ENONFINITE
        assert L.local_energy(ctypes.byref(m1), fake, ctypes.byref(H), 10, fake, fake, ws, 1 << 30, None) == \
            lib.VMC_ENONFINITE
        assert L.vmc_step(ctypes.byref(m1), fake, ctypes.byref(H), 10, 0, 0, None, None, fake, fake, None, fake,
                          fake, fake, ws, 1 << 30, None) == lib.VMC_ENONFINITE
    assert lib.VmcError(lib.VMC_ENONFINITE, "x").status == -5
    assert L.vmc_status_str(-5) == b"non-finite value"
    # 1D-only kinds on a lattice; negative exponent; a cluster chain needs n >= 3
    for H in (lib.ham(lib.VMC_LRTFIM, 1.0, 1.0, alpha=1.0), lib.ham(lib.VMC_CLUSTER, 1.0)):
        assert L.vmc_workspace_size(ctypes.byref(m2), ctypes.byref(H), 10, ctypes.byref(out)) == \
            lib.VMC_EUNSUPPORTED
    H = lib.ham(lib.VMC_LRTFIM, 1.0, 1.0, alpha=-0.5)
    assert L.vmc_workspace_size(ctypes.byref(m1), ctypes.byref(H), 10, ctypes.byref(out)) == lib.VMC_EINVAL
    H = lib.ham(lib.VMC_CLUSTER, 1.0)
    m_2 = lib.model(dims=1, Lx=2, d_h=16)
    assert L.vmc_workspace_size(ctypes.byref(m_2), ctypes.byref(H), 10, ctypes.byref(out)) == lib.VMC_EINVAL
    for n in (3, 12):
        m = lib.model(dims=1, Lx=n, d_h=16)
        assert L.vmc_workspace_size(ctypes.byref(m), ctypes.byref(H), 10, ctypes.byref(out)) == 0
    # grow_hidden noise
    assert L.grow_hidden(ctypes.byref(m1), fake, 32, 0, inf, fake, None, None, None, None, None) == lib.VMC_ENONFINITE
    assert L.grow_hidden(ctypes.byref(m1), fake, 32, 0, nan, fake, None, None, None, None, None) == lib.VMC_ENONFINITE
    # Adam settings
    t = ctypes.c_void_p(0x300000)
    for cfg, want in ((lib.adam_cfg(lr0=nan), lib.VMC_ENONFINITE), (lib.adam_cfg(eps=inf), lib.VMC_ENONFINITE),
                      (lib.adam_cfg(beta1=1.0), lib.VMC_EINVAL), (lib.adam_cfg(eps=0.0), lib.VMC_EINVAL),
                      (lib.adam_cfg(lr0=-1e-3), lib.VMC_EINVAL), (lib.adam_cfg(tau=-1.0), lib.VMC_EINVAL)):
        assert L.vmc_adam(100, fake, fake, fake, fake, t, ctypes.byref(cfg), None) == want
    assert L.vmc_adam(0, fake, fake, fake, fake, t, ctypes.byref(lib.adam_cfg()), None) == lib.VMC_EINVAL
    # the synchronous finiteness check validates its workspace first
    assert L.vmc_check_finite(fake, 10, None, ws, 255, None) == lib.VMC_EINVAL
    assert L.vmc_check_finite(fake, 10, None, ctypes.c_void_p(0x200010), 1024, None) == lib.VMC_EINVAL


def test_workspace_grows_with_samples(lib):
    m = lib.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True, precision=lib.VMC_BF16)
    H = lib.ham(lib.VMC_TFIM, 1.0, 3.0)
    a, b = lib.workspace_size(m, H, 1000), lib.workspace_size(m, H, 10000)
    assert b > 5 * a
    Hh = lib.ham(lib.VMC_HEISENBERG, 1.0, 0.0, True)
    assert lib.workspace_size(m, Hh, 1000) >= a


def test_tuning_table(lib):
    """Row-tile options, set/get/reset of the tuning table and its argument
    checks (host-only calls); the workspace size does not depend on it."""
    m = lib.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True, precision=lib.VMC_BF16)
    H = lib.ham(lib.VMC_TFIM, 1.0, 3.0)
    assert lib.row_tile_options(m) == [64, 48]
    builtin = lib.get_tuning(m)  # the chain default comes from the occupancy query (2 without a GPU)
    assert builtin["row_tile"] == 64 and 1 <= builtin["chain_wgs_per_cu"] <= 4
    # the 1D model of the same width starts from the shorter tile
    assert lib.row_tile_options(lib.model(dims=1, Lx=20, d_h=128, precision=lib.VMC_BF16)) == [48, 64]
    need = lib.workspace_size(m, H, 10000)
    lib.set_tuning(m, row_tile=48, chain_wgs_per_cu=4)
    try:
        assert lib.get_tuning(m) == {"row_tile": 48, "chain_wgs_per_cu": 4}
        assert lib.workspace_size(m, H, 10000) == need
        # another shape is untouched
        m2 = lib.model(dims=2, Lx=10, Ly=10, d_h=128, glu=True, precision=lib.VMC_FP32)
        assert lib.get_tuning(m2)["row_tile"] == 32
        assert lib.row_tile_options(m2) == [32, 16]
        for bad in [dict(row_tile=40), dict(chain_wgs_per_cu=5), dict(chain_wgs_per_cu=-1)]:
            with pytest.raises(lib.VmcError) as e:
                lib.set_tuning(m, **bad)
            assert e.value.status == -1
        # a rejected call leaves the table as it was
        assert lib.get_tuning(m) == {"row_tile": 48, "chain_wgs_per_cu": 4}
    finally:
        lib.reset_tuning(m)
    assert lib.get_tuning(m) == builtin
    # shapes without an alternative tile: one option
    m3 = lib.model(dims=1, Lx=20, d_h=16, precision=lib.VMC_BF16)
    assert lib.row_tile_options(m3) == [64]
    # the tuning cache file round trip
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tuning.json")
        lib.set_tuning(m, row_tile=48, chain_wgs_per_cu=1)
        lib.save_tuning(path, [m, m3])
        lib.reset_tuning(m)
        assert lib.load_tuning(path, [m, m3]) == 2
        assert lib.get_tuning(m) == {"row_tile": 48, "chain_wgs_per_cu": 1}
        lib.reset_tuning(m)
        lib.reset_tuning(m3)


def test_lds_size_limits(lib):
    """A model whose tiles do not fit the 160 KiB LDS of a compute unit is
    refused as unsupported, by the workspace query and by every entry point,
    before any device pointer is touched: bfloat16 d_h = 128 takes 2D lattices
    up to 29x29, d_h = 256 up to 24x24."""
    L = lib.lib()
    out = ctypes.c_size_t(0)
    for dh, ok in ((128, 29), (256, 24)):
        m = lib.model(dims=2, Lx=ok, Ly=ok, d_h=dh, glu=True, precision=lib.VMC_BF16)
        assert L.vmc_workspace_size(ctypes.byref(m), None, 10, ctypes.byref(out)) == 0
        m = lib.model(dims=2, Lx=ok + 1, Ly=ok + 1, d_h=dh, glu=True, precision=lib.VMC_BF16)
        assert L.vmc_workspace_size(ctypes.byref(m), None, 10, ctypes.byref(out)) == -2
        fake = ctypes.c_void_p(0x100000)
        ws = ctypes.c_void_p(0x200000)
        assert L.rnn_logpsi(ctypes.byref(m), fake, 10, fake, fake, None, ws, 1 << 40, None) == -2
        H = lib.ham(lib.VMC_TFIM, 1.0, 1.0)
        assert L.local_energy(ctypes.byref(m), fake, ctypes.byref(H), 10, fake, fake, ws, 1 << 40, None) == -2
    # 1D chains up to N = 1024 at every width
    m = lib.model(dims=1, Lx=1024, d_h=256, glu=True, precision=lib.VMC_BF16)
    assert L.vmc_workspace_size(ctypes.byref(m), None, 10, ctypes.byref(out)) == 0
