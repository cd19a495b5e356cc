"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side parameter derivation agrees with the oracle's own
derivation and with the definitions of the dimensionless groups."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import params as oparams
from paper_2110_05943_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="clb.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2110_05943_amd import nn
    lib = C.CDLL(B.LIB_PATH)
    names = declared_functions("clb.h")
    nn_names = declared_functions("clb_nn.h")
    assert len(names) >= 20 and len(nn_names) >= 16
    for n in names + nn_names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)
    assert set(nn_names) == set(nn.NN_EXPORTS)


def test_struct_sizes_match_header_layout(tmp_path):
    # The ctypes mirrors must have the C compiler's size and field offsets.
    fields = ("nx", "bc_u", "inlet_U", "eps", "scaling", "u_ref", "a", "gbeta", "T_init",
              "storage", "model", "a_rows", "forcing")
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"clb.h\"\nint main(void) {\n"
                   '  printf("%zu %zu\\n", sizeof(clb_params), sizeof(clb_derived));\n' +
                   "".join('  printf("%%zu\\n", offsetof(clb_params, %s));\n' % f for f in fields) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == C.sizeof(B.Params) and int(out[1]) == C.sizeof(B.Derived)
    for f, off in zip(fields, out[2:]):
        assert getattr(B.Params, f).offset == int(off), f


def test_create_rejects_non_finite_row_acceleration():
    lib = B._lib()
    rows = [0.0, 1e-5] * 7 + [0.0, float("nan")]
    p = B.make_params(nx=8, ny=8, bc=("periodic", "periodic", "wall_T", "wall_T"), Ra=1e3,
                      Pr=1.0, a_rows=rows)
    ctx = C.c_void_p()
    # rejected before the workspace is looked at
    assert lib.clb_create(C.byref(p), 1, None, 16, None, C.byref(ctx)) == B.ERR_ARG
    p = B.make_params(nx=8, ny=8, bc=("periodic", "periodic", "wall_T", "wall_T"), Ra=1e3,
                      Pr=1.0, a_rows=[0.0, 1e-5] * 8)
    assert lib.clb_create(C.byref(p), 1, None, 16, None, C.byref(ctx)) == B.ERR_WORKSPACE
    n8 = C.c_size_t(0)
    n0 = C.c_size_t(0)
    assert lib.clb_workspace_bytes(C.byref(p), 1, C.byref(n8)) == B.OK
    p.a_rows = None
    assert lib.clb_workspace_bytes(C.byref(p), 1, C.byref(n0)) == B.OK
    assert n8.value == n0.value + 256  # 16 doubles, one aligned block


@pytest.mark.parametrize("n,Ra,Pr,Da,phi", [(64, 1e3, 1.0, 1e-2, 0.6), (128, 1e5, 0.71, 1e-4, 0.4),
                                            (512, 1e7, 7.0, 1e-5, 0.95)])
def test_cavity_derivation_matches_oracle(n, Ra, Pr, Da, phi):
    d = B.derive(nx=n, ny=n, Ra=Ra, Pr=Pr, Da=Da, phi=phi, F_phi=-1.0)
    o = oparams.cavity(n, Ra=Ra, Pr=Pr, Da=Da, phi=phi)
    assert math.isclose(d["s_v"], o["s_v"], rel_tol=1e-14)
    assert math.isclose(d["zeta_a"], o["za"], rel_tol=1e-14)
    assert math.isclose(d["nu"], o["nu"], rel_tol=1e-14)
    assert math.isclose(d["gbeta"], o["gbeta_dT"], rel_tol=1e-14)
    assert math.isclose(d["K"], o["K"], rel_tol=1e-14)
    assert math.isclose(d["F_phi"], o["Fphi"], rel_tol=1e-14)
    assert d["L"] == n - 1
    # paper defaults (Section 3)
    assert (d["s1"], d["s3"], d["s4"], d["zeta_e"], d["zeta_nu"], d["varpi"]) == \
        (1.0, 1.2, 1.8, 1.0, 1.0, 0.25)
    assert d["s_b"] == 1.5


def test_channel_derivation_matches_oracle():
    ny, Re, u1 = 33, 5.0, 5.0 / 6.0 / 32
    d = B.derive(nx=4, ny=ny, bc=("periodic", "periodic", "wall_T", "wall_T"), scaling="channel",
                 Re=Re, u_ref=u1, Ra=100.0, Pr=1.0, Da=0.01, phi=0.6)
    o = oparams.channel(ny, Re=Re, Ra=100.0, Pr=1.0, Da=0.01, phi=0.6, u_ref=u1)
    for a, b in (("s_v", "s_v"), ("zeta_a", "za"), ("nu", "nu"), ("gbeta", "gbeta_dT"),
                 ("K", "K")):
        assert math.isclose(d[a], o[b], rel_tol=1e-13), a
    assert math.isclose(d["s_v"], 1.0, rel_tol=1e-13)


@pytest.mark.parametrize("bad", [dict(nx=3), dict(phi=0.0), dict(phi=1.5), dict(s_v=2.5),
                                 dict(bc=("periodic", "wall_T", "wall_T", "wall_T")),
                                 dict(Ra=0.0), dict(varpi=1.2), dict(storage=7)])
def test_invalid_parameters_are_rejected(bad):
    kw = dict(nx=16, ny=16, Ra=1e3, Pr=1.0, Da=1e-2, phi=0.6)
    kw.update(bad)
    with pytest.raises(B.CLBError) as e:
        B.derive(**kw)
    assert e.value.status == B.ERR_ARG


def test_workspace_bytes():
    lib = B._lib()
    arr = (B.Params * 2)(B.make_params(nx=64, ny=64, Ra=1e3, Pr=1.0),
                         B.make_params(nx=100, ny=30, Ra=1e3, Pr=1.0))
    n = C.c_size_t()
    assert lib.clb_workspace_bytes(arr, 2, C.byref(n)) == 0
    # two population buffers of 14 FP32 planes each per domain, rows padded to 64
    assert n.value > 2 * 14 * 4 * (64 * 64 + 128 * 30)
    arr[1].storage = 1
    assert lib.clb_workspace_bytes(arr, 2, C.byref(n)) == B.ERR_ARG  # storage must agree
    # FP32 planes with FP32 arithmetic: the same planes as FP32 storage
    arr[1].storage = 0
    assert lib.clb_workspace_bytes(arr, 2, C.byref(n)) == 0
    f32 = n.value
    arr[0].storage = arr[1].storage = B.STORE_F32C
    assert lib.clb_workspace_bytes(arr, 2, C.byref(n)) == 0 and n.value == f32


def test_create_rejects_small_workspace():
    lib = B._lib()
    p = B.make_params(nx=64, ny=64, Ra=1e3, Pr=1.0)
    ctx = C.c_void_p()
    # a too-small (and null) workspace fails before any device call
    assert lib.clb_create(C.byref(p), 1, None, 16, None, C.byref(ctx)) == B.ERR_WORKSPACE


def test_calls_without_context_are_rejected():
    lib = B._lib()
    steps = (C.c_int64 * 1)()
    status = (C.c_int32 * 1)()
    assert lib.clb_run(None, 100, 10, 1e-8, -1, None, 0, steps, status) == B.ERR_ARG
    assert lib.clb_step(None, 1) == B.ERR_ARG
    assert lib.clb_set_active(None, None) == B.ERR_ARG
    assert lib.clb_strerror(B.NOT_CONVERGED).decode() == "not steady within the step limit"


def test_network_calls_validate_arguments_on_the_host():
    """Invalid sizes, pointers or alignment are rejected before any launch."""
    from paper_2110_05943_amd import nn
    lib = nn.lib()
    vp = C.c_void_p
    a16 = vp(4096)  # aligned, never dereferenced: the call fails validation first
    bad = vp(4098)
    # channel counts must be multiples of 16; pointers 16-byte aligned
    assert lib.clb_nn_conv3x3(a16, 1, 4, 4, 8, a16, None, 16, 0, 0.0, a16, 1, None) == B.ERR_ARG
    assert lib.clb_nn_conv3x3(a16, 1, 4, 4, 16, a16, None, 24, 0, 0.0, a16, 1, None) == B.ERR_ARG
    assert lib.clb_nn_conv3x3(bad, 1, 4, 4, 16, a16, None, 16, 0, 0.0, a16, 1, None) == B.ERR_ARG
    assert lib.clb_nn_conv3x3(a16, 0, 4, 4, 16, a16, None, 16, 0, 0.0, a16, 1, None) == B.ERR_ARG
    assert lib.clb_nn_pool2(a16, 1, 5, 4, 16, a16, None) == B.ERR_ARG  # odd height
    assert lib.clb_nn_adamw(a16, a16, a16, a16, 10, 1e-3, 0.9, 0.999, 1e-8, 0.0, 0, None) \
        == B.ERR_ARG  # step t must be >= 1
    n = C.c_size_t()
    assert lib.clb_nn_wgrad_workspace_bytes(2, 16, 16, 16, 32, C.byref(n)) == B.OK
    assert n.value > 32 * 144 * 4
    assert lib.clb_nn_conv3x3_wgrad(a16, a16, 2, 16, 16, 16, 32, a16, None, a16, n.value - 4,
                                    None) == B.ERR_ARG  # workspace too small
    assert lib.clb_set_state_device(None, 0, a16, 16, 1.0, 0.0) == B.ERR_ARG
    co, ci = np.array([16, 0], dtype=np.int32), np.array([16, 16], dtype=np.int32)
    off = np.array([0, 4096], dtype=np.int64)
    tab = [t.ctypes.data_as(vp) for t in (co, ci, off)]
    assert lib.clb_nn_weights_bf16_layers(a16, 0, *tab, a16, a16, None) == B.ERR_ARG
    assert lib.clb_nn_weights_bf16_layers(a16, 65, *tab, a16, a16, None) == B.ERR_ARG
    assert lib.clb_nn_weights_bf16_layers(a16, 2, *tab, a16, a16, None) == B.ERR_ARG  # cout 0
    assert lib.clb_nn_mse(a16, 12, a16, 3, 10, a16, a16, a16, 1 << 20, None) == B.ERR_ARG
    desc = (np.array([16, 16], dtype=np.int32), np.array([16, 16], dtype=np.int32),
            np.array([2320, 0], dtype=np.int64))  # offsets must increase
    dtab = [t.ctypes.data_as(vp) for t in desc]
    assert lib.clb_nn_adamw_layers(a16, a16, a16, a16, 10000, 1e-3, 0.9, 0.999, 1e-8, 0.0, 1, 2,
                                   *dtab, a16, a16, None) == B.ERR_ARG
    ns = C.c_int32(0)
    assert lib.clb_nn_conv3x3_wgrad_parts(a16, a16, 2, 16, 16, 16, 32, 1, a16, n.value - 4,
                                          C.byref(ns), None) == B.ERR_ARG  # workspace too small
    assert lib.clb_nn_conv3x3_wgrad_parts(a16, a16, 2, 16, 16, 16, 32, 1, a16, n.value, None,
                                          None) == B.ERR_ARG  # no chunk count
    ptrs = (C.c_void_p * 2)(4096, None)
    one = (C.c_int32 * 2)(1, 1)
    assert lib.clb_nn_wgrad_reduce_layers(0, ptrs, one, one, one, ptrs, ptrs, None) == B.ERR_ARG
    assert lib.clb_nn_wgrad_reduce_layers(2, ptrs, one, one, one, ptrs, ptrs, None) == B.ERR_ARG


def test_bgk_derivation_uses_one_rate_per_lattice():
    d = B.derive(nx=64, ny=64, Ra=1e4, Pr=0.71, Da=1e-2, phi=0.6, model="bgk")
    assert d["s_b"] == d["s1"] == d["s3"] == d["s4"] == d["s_v"]
    assert d["zeta_e"] == d["zeta_nu"] == d["zeta_a"]
    m = B.derive(nx=64, ny=64, Ra=1e4, Pr=0.71, Da=1e-2, phi=0.6, model="mrt")
    assert (m["s_b"], m["s3"], m["s4"]) == (1.5, 1.2, 1.8)
    with pytest.raises(B.CLBError):
        B.derive(nx=64, ny=64, Ra=1e4, Pr=0.71, model=3)


def test_largest_domain_is_accepted_and_one_row_more_rejected():
    # 32-bit plane addressing: ny * pitch <= 2^30 elements
    ok = B.derive(nx=32768, ny=32768, Ra=1e6, Pr=1.0)
    assert ok["L"] == 32767
    with pytest.raises(B.CLBError):
        B.derive(nx=32768, ny=32769, Ra=1e6, Pr=1.0)
    with pytest.raises(B.CLBError):
        B.derive(nx=2 ** 31 - 1, ny=4, Ra=1e6, Pr=1.0)


def test_plane_offsets_are_64_bit_at_the_largest_domain():
    # The largest accepted FP32 domain has 2^30 elements per plane; the 14
    # population planes of a buffer then span offsets up to 13 * 2^30, and
    # the snapshot and observation planes up to 3 * 2^30, beyond INT32_MAX.
    # Every kernel forms plane offsets in 64-bit arithmetic: each product of
    # a plane count with `plane` in the kernel source is widened to size_t.
    d = B.derive(nx=32768, ny=32768, Ra=1e6, Pr=1.0)
    assert d["L"] == 32767
    plane = 32768 * 32768
    assert 13 * plane > 2 ** 31 - 1 and 2 * plane > 2 ** 31 - 1
    src = open(os.path.join(ROOT, "paper_2110_05943_amd", "csrc", "clb_kernels.hip")).read()
    src = re.sub(r"//[^\n]*", "", src)
    for m in re.finditer(r"(\S+)\s*\*\s*(d\.)?plane\b", src):
        pre = src[max(0, m.start() - 20):m.end()]
        assert "(size_t)" in pre, pre
    for m in re.finditer(r"\b(d\.)?plane\s*\+\s*idx", src):
        pre = src[max(0, m.start() - 20):m.end()]
        assert "(size_t)" in pre, pre
