"""The C-ABI library loads and exports every entry point include/mrcm.h
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mrcm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrcm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_call_set():
    names = declared_symbols()
    for required in ("mrcm_setup", "mrcm_update_mobility", "mrcm_solve", "mrcm_fine_flux",
                     "mrcm_destroy", "mrcm_last_error", "mrcm_get_stats"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2104_04653_amd import mrcm as binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmrcm.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTED) <= set(declared_symbols())


def test_null_arguments_rejected_without_gpu():
    """Argument validation happens before any device call."""
    from paper_2104_04653_amd import mrcm as binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmrcm.so not built")
    lib = binding.load_library()
    ctx = ctypes.c_void_p()
    rc = lib.mrcm_setup(ctypes.byref(ctx), None, None, 16, 16, 0, 2, 2, None, 1.0, None, None,
                        None, 0, None)
    assert rc == binding.E_INVAL
    assert lib.mrcm_solve(None) == binding.E_INVAL
    assert lib.mrcm_fine_flux(None, None, None, None, 0, None) == binding.E_INVAL
    lib.mrcm_destroy(None)


def test_bad_sizes_rejected_without_gpu():
    from paper_2104_04653_amd import mrcm as binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmrcm.so not built")
    import numpy as np
    lib = binding.load_library()
    grid = binding.Grid(60, 64, 1.0, 1.0)    # 60 is not a multiple of 16
    perm = np.ones(60 * 64)
    bc = binding.BC()
    for s in range(4):
        bc.kind[s] = 0
    fl = binding.Fluid(1.0, 10.0)
    ctx = ctypes.c_void_p()
    dp = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = lib.mrcm_setup(ctypes.byref(ctx), ctypes.byref(grid), dp, 16, 16, 0, 2, 2, None, 1.0,
                        ctypes.byref(bc), None, ctypes.byref(fl), 0, None)
    assert rc == binding.E_INVAL
    grid = binding.Grid(64, 64, 1.0, 1.0)
    perm = np.ones(64 * 64)
    perm[5] = -1.0
    dp = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = lib.mrcm_setup(ctypes.byref(ctx), ctypes.byref(grid), dp, 16, 16, 0, 2, 2, None, 1.0,
                        ctypes.byref(bc), None, ctypes.byref(fl), 0, None)
    assert rc == binding.E_INVAL
    perm[5] = 1.0
    rc = lib.mrcm_setup(ctypes.byref(ctx), ctypes.byref(grid), dp, 16, 16, 0, 3, 2, None, 1.0,
                        ctypes.byref(bc), None, ctypes.byref(fl), 0, None)
    assert rc == binding.E_INVAL            # linear spaces have 2 + 2 dofs
    rc = lib.mrcm_setup(ctypes.byref(ctx), ctypes.byref(grid), dp, 16, 16, 0, 2, 2, None, -1.0,
                        ctypes.byref(bc), None, ctypes.byref(fl), 0, None)
    assert rc == binding.E_INVAL            # alpha must be positive


def test_surrogate_entry_points_reject_null_without_gpu():
    from paper_2104_04653_amd import mrcm as binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmrcm.so not built")
    lib = binding.load_library()
    assert set(binding.EXPORTED) == set(declared_symbols())
    net = ctypes.c_void_p()
    assert lib.mrcm_cnn_create(None, 4, 0, None) == binding.E_INVAL
    assert lib.mrcm_cnn_create(ctypes.byref(net), 0, 0, None) == binding.E_INVAL
    assert lib.mrcm_cnn_num_params(None, None) == binding.E_INVAL
    assert lib.mrcm_cnn_forward(None, None, None, 1) == binding.E_INVAL
    assert lib.mrcm_cnn_loss_grad(None, None, None, 1, None, None) == binding.E_INVAL
    assert lib.mrcm_cnn_train_step(None, None, None, 1, 1e-3, None) == binding.E_INVAL
    assert lib.mrcm_set_surrogate(None, None) == binding.E_INVAL
    assert lib.mrcm_surrogate_inputs(None, None) == binding.E_INVAL
    assert lib.mrcm_surrogate_targets(None, None) == binding.E_INVAL
    assert lib.mrcm_solve_with_predictions(None, None) == binding.E_INVAL
    assert lib.mrcm_set_gate_tolerance(None, 1e-6) == binding.E_INVAL
    assert lib.mrcm_set_refinement(None, 8, 1e-9) == binding.E_INVAL
    assert lib.mrcm_set_interface_refinement(None, 3, 1e-14, 1e-10) == binding.E_INVAL
    lib.mrcm_cnn_destroy(None)


def test_binding_checks_alpha_length_without_gpu():
    """One Robin parameter per interface: a short array is rejected by the
    binding before the library could read past its end."""
    from paper_2104_04653_amd import mrcm as binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmrcm.so not built")
    import numpy as np
    import inputs
    prob = inputs.make_problem("gauss64", sub=16)           # 4 x 4 subdomains: 24 interfaces
    with pytest.raises(ValueError):
        binding.MRCMSolver(prob.replace(alpha_per_interface=np.ones(23)))


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (compiled here with gcc)."""
    import shutil
    import subprocess
    from paper_2104_04653_amd import mrcm as binding
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    pairs = {"mrcm_stats": binding.Stats, "mrcm_transport_stats": binding.TransportStats,
             "mrcm_sfi_stats": binding.SFIStats}
    for cname in ("Grid", "BC", "Fluid"):
        if hasattr(binding, cname):
            pairs[{"Grid": "mrcm_grid", "BC": "mrcm_bc", "Fluid": "mrcm_fluid"}[cname]] = getattr(binding, cname)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mrcm.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
