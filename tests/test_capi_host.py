"""Host-side checks of the C ABI library (no GPU needed).

The library loads, exports every function include/claw.h declares, its
descriptor struct matches the binding's layout, and descriptor validation
rejects bad input before any HIP call is made.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "claw.h")


@pytest.fixture(scope="module")
def claw():
    from paper_1805_08846_amd import claw as c
    return c


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(claw_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function(claw):
    lib = ctypes.CDLL(claw.library_path())
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in claw.h but not exported"
    assert sorted(claw.EXPORTED) == declared


def test_debug_library_exports_every_declared_function(claw):
    # the range-checked build (CLAW_DEBUG) has the same ABI
    path = os.path.join(ROOT, "paper_1805_08846_amd", "libclaw_debug.so")
    if not os.path.exists(path):
        pytest.skip("libclaw_debug.so not built")
    lib = ctypes.CDLL(path)
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in claw.h but not exported by the debug build"


def test_release_build_reports_no_range_checks(claw):
    with pytest.raises(claw.ClawError) as e:
        claw.claw_debug_take()
    assert e.value.status == claw.CLAW_E_UNSUPPORTED


@pytest.mark.parametrize("struct", ["claw_desc", "claw_lc_desc"])
def test_descriptor_layout_matches_header(claw, tmp_path, struct):
    cls = getattr(claw, struct)
    src = tmp_path / "layout.c"
    fields = [f for f, _ in cls._fields_]
    body = "\n".join(f'printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "claw.h"\nint main(void){\n'
                   + body + f'\nprintf("sizeof %zu\\n", sizeof({struct}));\nreturn 0;}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    for f in fields:
        assert int(got[f]) == getattr(cls, f).offset, f
    assert int(got["sizeof"]) == ctypes.sizeof(cls)


def _sw_desc(claw, n=64):
    d = claw.claw_desc_init()
    d.ndim = 2
    d.n[0] = d.n[1] = n
    d.n[2] = 1
    d.lower[0] = d.lower[1] = -1.0
    d.upper[0] = d.upper[1] = 1.0
    d.riemann = claw.CLAW_RP_SHALLOW_WATER
    d.meqn = d.mwaves = 3
    d.dtype = claw.CLAW_FP32
    return d


def test_workspace_size(claw):
    d = _sw_desc(claw, 64)
    nb = claw.claw_workspace_bytes(d)
    # two scratch state buffers plus the control block (step state and the
    # per-direction speed slots, 128 bytes each, page aligned)
    assert nb >= 2 * 3 * 64 * 64 * 4
    assert nb < 2 * 3 * 64 * 64 * 4 + 24 * 1024


@pytest.mark.parametrize("field,value", [
    ("ndim", 4), ("meqn", 4), ("num_ghost", 3), ("dtype", 7), ("limiter", 9),
    ("grav", -1.0), ("cfl_desired", 0.0), ("riemann", 5)])
def test_bad_descriptors_are_rejected(claw, field, value):
    d = _sw_desc(claw)
    setattr(d, field, value)
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status in (claw.CLAW_E_INVALID, claw.CLAW_E_UNSUPPORTED)
    assert claw.claw_last_error()


def test_bad_grid_and_bc(claw):
    d = _sw_desc(claw)
    d.n[0] = 0
    with pytest.raises(claw.ClawError):
        claw.claw_workspace_bytes(d)
    d = _sw_desc(claw)
    d.bc_lo[1] = 3
    with pytest.raises(claw.ClawError):
        claw.claw_workspace_bytes(d)
    d = _sw_desc(claw)
    d.ndim = 3
    d.n[2] = 4
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED


def test_grid_size_limits(claw):
    # extents whose product overflows 64 bits, and a grid just past the 32-bit
    # element offsets, are refused on the host; one just inside is accepted
    d = _sw_desc(claw)
    d.n[0] = 1 << 40
    d.n[1] = 1 << 40
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    d = _sw_desc(claw)
    d.n[0] = 1 << 16
    d.n[1] = (1 << 31) // (3 << 16) + 1
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    d.n[1] -= 1
    assert claw.claw_workspace_bytes(d) >= 2 * 3 * 4 * d.n[0] * d.n[1]


def test_batch_size_limits(claw):
    # a batched sweep is one launch of at most 2^24 - 1 workgroups: 300 grids
    # of 1 x 262140 cells need 300 x 65535 row workgroups and are refused;
    # 200 of them fit
    d = _sw_desc(claw)
    d.n[0], d.n[1] = 1, 65535 * 4
    with pytest.raises(claw.ClawError) as e:
        claw.claw_batch_workspace_bytes([d] * 300)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    assert claw.claw_batch_workspace_bytes([d] * 200) >= 2 * 3 * 4 * 200 * d.n[1]
    assert claw.claw_batch_workspace_bytes([_sw_desc(claw)] * 4) > 0


def test_batch_step_flags(claw):
    # a batch runs one kind of step: every instance split, or every instance
    # fused (the fused batch holds its workgroup table and per-instance
    # arguments in the workspace too); mixed or other flags are refused
    split = _sw_desc(claw)
    fused = _sw_desc(claw)
    fused.flags = claw.CLAW_FLAG_FUSED_STEP
    assert claw.claw_batch_workspace_bytes([fused] * 3) > claw.claw_batch_workspace_bytes([split] * 3)
    with pytest.raises(claw.ClawError) as e:
        claw.claw_batch_workspace_bytes([split, fused])
    assert e.value.status == claw.CLAW_E_INVALID
    # without flags a batch follows the single grid's rule on its whole
    # state: 4 x 3000^2 FP32 (432 MB) takes the fused step, 3 small grids not
    big = _sw_desc(claw)
    big.n[0] = big.n[1] = 3000
    big_fused = _sw_desc(claw)
    big_fused.n[0] = big_fused.n[1] = 3000
    big_fused.flags = claw.CLAW_FLAG_FUSED_STEP
    big_split = _sw_desc(claw)
    big_split.n[0] = big_split.n[1] = 3000
    big_split.flags = claw.CLAW_FLAG_SPLIT_STEP
    assert claw.claw_batch_workspace_bytes([big] * 4) == claw.claw_batch_workspace_bytes([big_fused] * 4)
    assert claw.claw_batch_workspace_bytes([big] * 4) > claw.claw_batch_workspace_bytes([big_split] * 4)
    assert claw.claw_batch_workspace_bytes([split] * 3) < claw.claw_batch_workspace_bytes([fused] * 3)
    with pytest.raises(claw.ClawError) as e:
        claw.claw_batch_workspace_bytes([big, big_split])
    assert e.value.status == claw.CLAW_E_INVALID
    strang = _sw_desc(claw)
    strang.flags = claw.CLAW_FLAG_STRANG
    with pytest.raises(claw.ClawError) as e:
        claw.claw_batch_workspace_bytes([strang])
    assert e.value.status == claw.CLAW_E_UNSUPPORTED


def _burgers_desc(claw, ndim=2):
    from paper_1805_08846_amd import inputs
    prob, _, _ = (inputs.burgers2d(n=32) if ndim == 2 else inputs.burgers3d(n=16))
    return claw.desc_from_problem(prob)


def test_plugin_descriptors(claw):
    for ndim in (2, 3):
        d = _burgers_desc(claw, ndim)
        assert d.riemann == claw.CLAW_RP_BURGERS and d.meqn == d.mwaves == 1
        # one field, two scratch buffers
        assert claw.claw_workspace_bytes(d) >= 2 * d.n[0] * d.n[1] * d.n[2] * 8
    for field, value in [("meqn", 3), ("mwaves", 2), ("maux", 2)]:
        d = _burgers_desc(claw)
        setattr(d, field, value)
        with pytest.raises(claw.ClawError) as e:
            claw.claw_workspace_bytes(d)
        assert e.value.status == claw.CLAW_E_INVALID
    d = _burgers_desc(claw)
    d.param[1] = float("nan")
    with pytest.raises(claw.ClawError):
        claw.claw_workspace_bytes(d)
    # the shallow-water plug-in runs in 2D only; unknown plug-in ids fail
    d = _sw_desc(claw)
    d.riemann = claw.CLAW_RP_SHALLOW_WATER_GENERIC
    d.param[0] = 1.0
    claw.claw_workspace_bytes(d)
    d.ndim = 3
    d.n[2] = 4
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    d = _sw_desc(claw)
    d.riemann = 40
    with pytest.raises(claw.ClawError):
        claw.claw_workspace_bytes(d)
    with pytest.raises(claw.ClawError):
        claw.claw_plugin_info(40)
    info = claw.claw_plugin_info(claw.CLAW_RP_BURGERS)
    assert info == {"meqn": 1, "mwaves": 1, "ndim_max": 3, "vec_field": -1, "name": "burgers"}


def test_create_rejects_null_buffers_before_touching_the_gpu(claw):
    d = _sw_desc(claw)
    h = ctypes.c_void_p(None)
    st = claw._lib.claw_create(ctypes.byref(d), None, None, None, 0, None, ctypes.byref(h))
    assert st == claw.CLAW_E_INVALID
    assert "q is NULL" in claw.claw_last_error()


def test_null_handle_calls(claw):
    for fn, args in [("claw_step", (None, 1.0, None)), ("claw_sync_state", (None,)),
                     ("claw_advance", (None, 1, 0.0, None, None))]:
        assert getattr(claw._lib, fn)(*args) == claw.CLAW_E_INVALID
    assert claw._lib.claw_destroy(None) == claw.CLAW_OK


def test_status_strings(claw):
    for s in range(7):
        assert claw.claw_status_string(s)


def _lc_desc(claw, nx=64, ny=48):
    from paper_1805_08846_amd import inputs
    return claw.lc_desc(nx, ny, inputs.lc_norm())


def test_learned_sizes_and_validation(claw):
    d = _lc_desc(claw)
    pb, wb = claw.claw_lc_sizes(d)
    assert pb >= 3 * 4 * claw.CLAW_LC_NPARAM + 2 * (64 * 16 + 64 * 64 + 16 * 64)
    # dF, dG, cell gradients, flags and at least one partial gradient
    assert wb >= 4 * 3 * (48 * 65 + 49 * 64 + 48 * 64) + 48 * 64 + 4 * claw.CLAW_LC_NPARAM
    for field, value in [("nx", 1), ("ny", 0), ("nx", 1 << 40)]:
        bad = _lc_desc(claw)
        setattr(bad, field, value)
        with pytest.raises(claw.ClawError):
            claw.claw_lc_sizes(bad)
    bad = _lc_desc(claw)
    bad.nx = bad.ny = 1 << 40  # the product overflows 64 bits
    with pytest.raises(claw.ClawError) as e:
        claw.claw_lc_sizes(bad)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    bad = _lc_desc(claw)
    bad.sd2[1] = 0.0
    with pytest.raises(claw.ClawError):
        claw.claw_lc_sizes(bad)


def test_learned_calls_reject_null_buffers_before_touching_the_gpu(claw):
    d = _lc_desc(claw)
    L = claw._lib
    assert L.claw_lc_init(None, None) == claw.CLAW_E_INVALID
    assert L.claw_lc_forward(ctypes.byref(d), None, None, None, None, None) == claw.CLAW_E_INVALID
    w = (ctypes.c_double * 3)(1, 1, 1)
    assert L.claw_lc_loss_grad(ctypes.byref(d), None, None, None, None, 0.1, 0.1, w, None, None, None,
                               None) == claw.CLAW_E_INVALID
    assert L.claw_lc_adam(None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == claw.CLAW_E_INVALID
    fake = ctypes.c_void_p(4096)  # never dereferenced: the step count is checked first
    assert L.claw_lc_adam(fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None) == claw.CLAW_E_INVALID
    assert "count from 1" in claw.claw_last_error()
    assert L.claw_lc_apply(ctypes.byref(d), None, None, None, None, 0.1, 0.1, 0.5, 0.01, None, None, None,
                           None, None) == claw.CLAW_E_INVALID
    assert L.claw_lc_coarsen(0, 4, fake, fake, None) == claw.CLAW_E_INVALID
    assert L.claw_lc_advance(None, ctypes.byref(d), None, 1, 0.1, 0.5, 0.01, None) == claw.CLAW_E_INVALID


def test_philox_helper_known_answers():
    # the test helper the noise kernel is checked against reproduces the
    # published known-answer vectors of Philox4x32-10
    from helpers import philox4x32_10
    cases = [((0, 0, 0, 0, 0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 6, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for args, want in cases:
        assert tuple(int(v) for v in philox4x32_10(*args)) == want


def test_learned_scales_host_call(claw):
    # residual energies (sum over 64 cells) -> output scales and loss weights
    r2 = (64 * 4e-6, 64 * 9e-6, 64 * 1e-6)
    s_out, w = claw.claw_lc_scales(r2, 64, 0.5, True)
    assert s_out[0] == pytest.approx(2e-3 / 0.5, rel=1e-6)
    assert s_out[1] == s_out[2] == pytest.approx(0.5 * (3e-3 + 1e-3) / 0.5, rel=1e-6)
    assert w == pytest.approx((1 / 4e-6, 1 / 9e-6, 1 / 1e-6), rel=1e-12)
    s0, _ = claw.claw_lc_scales(r2, 64, 0.5, False)
    assert s0[0] == 0.0
    # a field with no residual gets the floor 1e-30, not a division by zero
    _, w0 = claw.claw_lc_scales((0.0, 1.0, 1.0), 64, 0.5, True)
    assert w0[0] == pytest.approx(1e30)
    with pytest.raises(claw.ClawError):
        claw.claw_lc_scales((1.0, 1.0, 1.0), 0, 0.5, True)


def test_fp64_field_byte_limit(claw):
    # the sweeps address a field with 32-bit byte offsets: an FP64 field of
    # 32768 x 16385 cells (4 GiB + 256 KiB) is refused, the FP32 one fits
    d = _sw_desc(claw)
    d.n[0], d.n[1] = 32768, 16385
    assert claw.claw_workspace_bytes(d) > 0
    d.dtype = claw.CLAW_FP64
    with pytest.raises(claw.ClawError) as e:
        claw.claw_workspace_bytes(d)
    assert e.value.status == claw.CLAW_E_UNSUPPORTED
    assert "4 GiB" in claw.claw_last_error()


def test_noalloc_sweep_rejects_on_the_host(claw):
    # bad arguments and grids beyond the scratch limit fail before any HIP
    # call (the pointers below are never dereferenced)
    fake_a, fake_b, fake_aux = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    d = _sw_desc(claw)
    lib = claw._lib
    assert lib.claw_sweep_noalloc(ctypes.byref(d), None, fake_b, None, 0, 0.1, None, None) == claw.CLAW_E_INVALID
    assert lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_a, None, 0, 0.1, None, None) == claw.CLAW_E_INVALID
    assert lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_b, None, 2, 0.1, None, None) == claw.CLAW_E_INVALID
    assert lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_b, None, 0, -1.0, None, None) == claw.CLAW_E_INVALID
    d.flags = claw.CLAW_FLAG_STRANG
    assert lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_b, None, 0, 0.1, None, None) == claw.CLAW_E_INVALID
    # acoustics with per-cell coefficients: 2 ncell sizeof(real) bytes of
    # scratch; 1024^2 FP64 (16 MiB) fits the limit, one more row does not
    from paper_1805_08846_amd import inputs
    prob, _, _ = inputs.acoustics3d_layers(n=8, dtype="f64", nsteps=1)
    d = claw.desc_from_problem(prob)
    assert d.maux == 2
    d.ndim, d.meqn = 2, 3
    d.n[0], d.n[1], d.n[2] = 1024, 1025, 1
    assert lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_b, None, 0, 0.1, None, None) == claw.CLAW_E_INVALID
    st = lib.claw_sweep_noalloc(ctypes.byref(d), fake_a, fake_b, fake_aux, 0, 0.1, None, None)
    assert st == claw.CLAW_E_UNSUPPORTED
    assert "scratch limit" in claw.claw_last_error()
