"""The C ABI boundary, checked on the host (no GPU): the library loads, exports every
entry point include/mppi.h declares, its structs have the documented layout, and the
host-side argument checks return the documented codes."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mppi.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:mppi_status|const char \*|double)\s*(mppi_\w+)\(", text, re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("mppi_create", "mppi_destroy", "mppi_reserve", "mppi_update", "mppi_rollout",
                 "mppi_weights", "mppi_weighted_sum", "mppi_apply_shift", "mppi_noise",
                 "mppi_philox", "mppi_plant_step", "mppi_validate", "mppi_status_str",
                 "mppi_last_error", "mppi_profile_enable", "mppi_profile_read"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2407_09812_amd as lib
    so = C.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(so, name), name
    assert set(lib.exported_symbols()) == set(declared_functions())
    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                             text=True, check=True).stdout
        exported = set(re.findall(r"\bT (mppi_\w+)$", out, re.M))
        assert set(declared_functions()) <= exported


def test_struct_layouts():
    import paper_2407_09812_amd as lib
    assert C.sizeof(lib.Vehicle) == 13 * 4
    assert C.sizeof(lib.Cost) == 15 * 4
    assert C.sizeof(lib.Solve) == 72 and lib.Solve.seed.offset == 48 and lib.Solve.dt_ctrl.offset == 64
    assert C.sizeof(lib.Diag) == 32
    assert lib.OBSTACLE_DTYPE.itemsize == 20


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layouts_match_the_c_header(tmp_path):
    """sizeof / offsetof of every ABI struct, compiled from include/mppi.h, equal the
    binding's ctypes layouts."""
    import paper_2407_09812_amd as lib
    structs = {"mppi_vehicle": lib.Vehicle, "mppi_cost": lib.Cost, "mppi_solve": lib.Solve,
               "mppi_diag": lib.Diag, "mppi_launch_config": lib.LaunchConfig,
               "mppi_request": lib.Request, "mppi_batch_config": lib.BatchConfig,
               "mppi_profile": lib.Profile, "mppi_server_cfg": lib.ServerCfg,
               "mppi_server_request": lib.ServerRequest, "mppi_server_result": lib.ServerResult,
               "mppi_server_stats": lib.ServerStats}
    c_name = {"lam": "lambda"}            # ctypes cannot name a field after a Python keyword
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mppi.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {c_name.get(f, f)}));')
    lines.append('printf("mppi_obstacle %zu\\n", sizeof(mppi_obstacle)); return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.strip().split("\n"))
    for cname, ct in structs.items():
        assert int(got[cname]) == C.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(ct, f).offset, (cname, f)
    assert int(got["mppi_obstacle"]) == lib.OBSTACLE_DTYPE.itemsize


def test_server_rejects_bad_configuration_on_the_host():
    import paper_2407_09812_amd as lib
    import workloads as W
    veh, cost = W.vehicle_benchmark(), W.cost_benchmark()
    for kw in (dict(n_vehicles=0), dict(N_max=5000), dict(n_streams=0), dict(max_batch=0),
               dict(budget_bytes=0), dict(M_max=-1)):
        args = dict(n_vehicles=4, K_max=256, N_max=50, M_max=10, n_streams=2, max_batch=8,
                    budget_bytes=1 << 24)
        args.update(kw)
        with pytest.raises(lib.MPPIError) as e:
            lib.Server(veh, cost, W.hover_control(veh), **args)
        assert e.value.status == -1
    with pytest.raises(lib.MPPIError) as e:
        lib.Server(dict(veh, mass=-1.0), cost, W.hover_control(veh), n_vehicles=4, K_max=256,
                   N_max=50, M_max=10)
    assert e.value.status == -1


def _good():
    sc = W.c2_line(K=128, N=10)
    return sc.veh, sc.cost, sc.solve(0)


@pytest.mark.parametrize("field,value,code", [
    ("K", 0, -1), ("N", 0, -1), ("N", 4097, -1), ("dt", 0.0, -1), ("dt", -1.0, -1),
    ("lam", 0.0, -1), ("lam", -2.0, -1), ("lam", float("nan"), -2), ("dt", float("inf"), -2),
])
def test_validate_solve_codes(field, value, code):
    import paper_2407_09812_amd as lib
    veh, cost, solve = _good()
    assert lib.mppi_validate(veh, cost, solve, 20) == 0
    solve[field] = value
    assert lib.mppi_validate(veh, cost, solve, 20) == code


def test_validate_other_codes():
    import paper_2407_09812_amd as lib
    veh, cost, solve = _good()
    assert lib.mppi_validate(veh, cost, solve, -1) == -1
    assert lib.mppi_validate(veh, cost, solve, lib.M_MAX + 1) == -1
    s2 = dict(solve, sigma=np.array([1.0, -0.1, 1.0, 1.0]))
    assert lib.mppi_validate(veh, cost, s2, 0) == -1
    for k, v, code in (("mass", 0.0, -1), ("T_min", 9.0, -1), ("tau_m", -0.01, -1),
                       ("g", float("nan"), -2)):
        assert lib.mppi_validate(dict(veh, **{k: v}), cost, solve, 0) == code
    assert lib.mppi_validate(veh, dict(cost, c_p=-1.0), solve, 0) == -1
    assert lib.mppi_validate(veh, dict(cost, obs_w=float("inf")), solve, 0) == -2


def test_null_context_is_rejected_without_device_access():
    import paper_2407_09812_amd as lib
    f = lib._lib
    assert f.mppi_update(None, None, None, None, None, None, None, None, 0, None, None, None) == -1
    assert f.mppi_reserve(None, 1, 1, 0) == -1
    assert f.mppi_destroy(None) == -1
    assert f.mppi_last_error(None) == b"null context"
    assert lib.mppi_status_str(-8) == "MPPI_E_CAPACITY"
    assert lib.mppi_status_str(0) == "MPPI_OK"
    out = C.c_void_p()
    assert f.mppi_device_address(None, C.byref(out)) == -1
    assert f.mppi_device_address(C.c_void_p(16), None) == -1


def test_binding_refuses_pageable_host_tensors():
    """Outputs may be device tensors or pinned host tensors (reached through their
    device address); pageable host memory is refused before any call."""
    import torch
    import paper_2407_09812_amd as lib
    with pytest.raises(ValueError):
        lib._ptr(torch.zeros(8))
    with pytest.raises(ValueError):
        lib._ptr(torch.zeros(8, 2).t())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_plain_c_program_links_the_abi(tmp_path):
    """The header is plain C and the library links into a C program."""
    import paper_2407_09812_amd as lib
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stdio.h>
#include "mppi.h"
int main(void) {
    mppi_vehicle v = {1.0f, {0.01f, 0.01f, 0.02f}, 0.15f, 0.012f, 9.81f, 0.0f, 8.0f,
                      0.03f, 0.0f, 0.0f, 0.0f};
    mppi_cost c = {400, 40, 20, 20, {0.01f, 0.05f, 0.05f, 0.1f}, {0.05f, 0.1f, 0.1f, 0.3f},
                   0.3f, 1000.0f, 1.0e4f};
    mppi_solve s = {256, 20, 0.01f, 1.0f, {1, 1, 1, 1}, {9.81f, 0, 0, 0}, 0, 0, 0};
    int ok = mppi_validate(&v, &c, &s, 0);
    s.lambda = 0.0f;
    int bad = mppi_validate(&v, &c, &s, 0);
    printf("%d %d %s\n", ok, bad, mppi_status_str(bad));
    return 0;
}
''')
    exe = tmp_path / "probe"
    libdir = os.path.dirname(lib.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-o", str(exe), str(src), "-L", libdir, "-lmppi", f"-Wl,-rpath,{libdir}"],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert out == ["0", "-1", "MPPI_E_INVALID_ARG"]
