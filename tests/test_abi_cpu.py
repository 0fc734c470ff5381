"""C-ABI checks that need no GPU: the library loads, exports every symbol the header
declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_1411_6206_amd as pls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prior_ls.h")

pytestmark = pytest.mark.skipif(not os.path.exists(pls.LIB_PATH),
                                reason="libprior_ls.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prior_ls_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(pls.EXPORTS)


def test_every_declared_symbol_is_exported():
    L = C.CDLL(pls.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_sizes_match_header():
    # offsets and sizes the C compiler assigns (x86-64 SysV)
    assert C.sizeof(pls.Dims) == 48
    assert C.sizeof(pls.Params) == 56
    assert C.sizeof(pls.Inputs) == 56
    assert C.sizeof(pls.Outputs) == 32
    assert C.sizeof(pls.Stats) == 8 + 24 + 6 * 8 + 64 * 8 + 8


def test_struct_layouts_match_a_c_compiler(tmp_path):
    # sizeof and the offset of the last field of every ABI struct, as gcc lays them out
    structs = {"prior_ls_dims": pls.Dims, "prior_ls_params": pls.Params,
               "prior_ls_inputs": pls.Inputs, "prior_ls_outputs": pls.Outputs,
               "prior_ls_stats": pls.Stats, "prior_ls_server_config": pls.ServerConfig,
               "prior_ls_request": pls.Request, "prior_ls_result": pls.Result,
               "prior_ls_server_stats": pls.ServerStats, "prior_ls_tuning": pls.Tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "prior_ls.h"', 'int main(void) {']
    for cname, py in structs.items():
        last = py._fields_[-1][0]
        lines.append(f'  printf("{cname} %zu %zu\\n", sizeof({cname}), offsetof({cname}, {last}));')
    lines.append('  return 0; }')
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        cname, size, off = line.split()
        py = structs[cname]
        assert C.sizeof(py) == int(size), cname
        assert getattr(py, py._fields_[-1][0]).offset == int(off), cname


def test_null_server_and_append_calls():
    L = pls.lib()
    L.prior_ls_server_destroy(None)
    assert L.prior_ls_append(None, None, None, None, None, None) == pls.EINVAL
    assert L.prior_ls_server_create(None, None) == pls.EINVAL
    s = C.c_void_p()
    assert L.prior_ls_server_create(None, C.byref(s)) == pls.EINVAL
    bad = pls.ServerConfig(C.sizeof(pls.ServerConfig), 0, 0, 0)       # max_active 0
    assert L.prior_ls_server_create(C.byref(bad), C.byref(s)) == pls.EINVAL
    bad = pls.ServerConfig(C.sizeof(pls.ServerConfig) + 1, 0, 1, 0)   # struct_size
    assert L.prior_ls_server_create(C.byref(bad), C.byref(s)) == pls.EINVAL
    t = C.c_int64()
    assert L.prior_ls_server_submit(None, None, C.byref(t)) == pls.EINVAL
    r = pls.Result()
    r.struct_size = C.sizeof(pls.Result)
    assert L.prior_ls_server_wait(None, 1, C.byref(r)) == pls.EINVAL
    st = pls.ServerStats()
    st.struct_size = C.sizeof(pls.ServerStats)
    assert L.prior_ls_server_info(None, C.byref(st)) == pls.EINVAL


def test_null_batch_calls():
    L = pls.lib()
    L.prior_ls_batch_destroy(None)
    assert L.prior_ls_batch_last_error(None) == b""
    b = C.c_void_p()
    assert L.prior_ls_batch_create(None, 1, C.byref(b)) == pls.EINVAL
    assert b.value is None
    arr = (C.c_void_p * 1)(None)
    assert L.prior_ls_batch_create(arr, 1, C.byref(b)) == pls.EINVAL      # NULL handle
    assert L.prior_ls_batch_create(arr, 0, C.byref(b)) == pls.EINVAL      # count 0
    assert L.prior_ls_batch_create(arr, 1, None) == pls.EINVAL
    assert L.prior_ls_batch_solve(None, None, None, None, None) == pls.EINVAL
    assert L.prior_ls_batch_step(None, 1, None, None) == pls.EINVAL


def test_server_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pls.PriorLSError) as e:
        pls.Server(max_active=2)
    assert e.value.status == pls.EHIP


def _create(**kw):
    base = dict(nx=64, ny=64, nz=1, nt=16, nc=1, wavelet_levels=2)
    base.update(kw)
    d = pls.make_dims(**base)
    h = C.c_void_p()
    rc = pls.lib().prior_ls_create(C.byref(d), None, C.byref(h))
    return rc, h, pls.lib().prior_ls_last_error(None).decode()


@pytest.mark.parametrize("kw,code", [
    (dict(nt=65), pls.ESHAPE),
    (dict(nt=33, transform="tfft"), pls.ESHAPE),   # the temporal transform takes <= 32 frames
    (dict(nt=0), pls.ESHAPE),
    (dict(ny=20), pls.ESHAPE),            # not in the FFT length set
    (dict(ny=512), pls.ESHAPE),
    (dict(nz=2), pls.ESHAPE),
    (dict(nx=100), pls.ESHAPE),
    (dict(wavelet_levels=4), pls.ESHAPE),
    (dict(wavelet_levels=-1), pls.ESHAPE),
    (dict(nz=4, wavelet_levels=3), pls.ESHAPE),   # 4 not divisible by 8
    (dict(nc=65), pls.ESHAPE),
    (dict(gram_mode=7), pls.EINVAL),
])
def test_create_rejects_bad_dims(kw, code):
    rc, h, msg = _create(**kw)
    assert rc == code, msg
    assert h.value is None
    assert msg


def test_create_rejects_null_and_size_mismatch():
    L = pls.lib()
    h = C.c_void_p()
    assert L.prior_ls_create(None, None, C.byref(h)) == pls.EINVAL
    d = pls.make_dims(64, 64, 1, 16, 1)
    d.struct_size = 12
    assert L.prior_ls_create(C.byref(d), None, C.byref(h)) == pls.EINVAL
    d = pls.make_dims(64, 64, 1, 16, 1)
    d.transform = 7                                   # unknown transform
    assert L.prior_ls_create(C.byref(d), None, C.byref(h)) == pls.EINVAL
    assert L.prior_ls_create(C.byref(pls.make_dims(64, 64, 1, 16, 1)), None, None) == pls.EINVAL


def test_budget_below_plan_is_enomem():
    need = pls.plan_bytes(64, 64, 1, 16, 1)
    assert need > 5 * 64 * 64 * 16 * 8
    rc, h, msg = _create(hbm_budget=need // 2)
    assert rc == pls.ENOMEM, msg


def test_temporal_transform_ignores_the_haar_divisibility():
    # nz = 4 with J = 3 is invalid for Haar, valid for the temporal transform
    assert pls.plan_bytes(16, 16, 4, 6, 2, wavelet_levels=3) == 0
    assert pls.plan_bytes(16, 16, 4, 6, 2, wavelet_levels=3, transform="tfft") > 0


def test_plan_bytes_zero_for_invalid():
    assert pls.plan_bytes(64, 64, 1, 65, 1) == 0
    assert pls.plan_bytes(64, 64, 1, 40, 1, transform="tfft") == 0


def test_windows_of_up_to_64_frames_are_accepted():
    # the wide Gram, the 64-frame eigensolver and back-projection operand: every transform
    # but the temporal one
    for nt in (33, 48, 64):
        assert pls.plan_bytes(64, 64, 1, nt, 1) > pls.plan_bytes(64, 64, 1, 32, 1)
        assert pls.plan_bytes(32, 32, 8, nt, 2, transform="db4") > 0


def test_null_handle_calls():
    L = pls.lib()
    L.prior_ls_destroy(None)
    assert L.prior_ls_step(None, 1, None, None) == pls.EINVAL
    assert L.prior_ls_solve(None, None, None, None, None) == pls.EINVAL
    assert L.prior_ls_op_dc(None, None, None, None) == pls.EINVAL
    for code in (0, -1, -2, -3, -4, -5):
        assert pls.strerror(code)
    assert pls.strerror(123) == "unknown status"


def test_valid_dims_without_gpu_fail_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h, msg = _create()
    assert rc == pls.EHIP
    assert h.value is None


def test_accepted_shapes_are_exactly_the_advertised_instances():
    # the (ny, nz) planes and readout lengths create accepts are the instances the parity
    # sweep (tests/test_gpu_sweep.py) compares with the oracle, no more and no fewer
    from instances import PLANES, READOUT_NX
    acc = {(ny, nz) for ny in range(1, 300) for nz in range(1, 40)
           if pls.plan_bytes(16, ny, nz, 3, 2, wavelet_levels=0) > 0}
    assert acc == set(PLANES)
    acc_x = {nx for nx in range(1, 300) if pls.plan_bytes(nx, 16, 4, 3, 2, wavelet_levels=0) > 0}
    assert acc_x == set(READOUT_NX)
    assert len(PLANES) == 50
