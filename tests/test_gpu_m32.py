"""32 x 32 subdomains on the GPU (the 2048 x 1024 channelized workload with
edge-solution interface spaces, and smaller cases of the same shape),
against the oracle at relative L2 1e-10 in pressure and flux."""
import numpy as np
import pytest

import inputs
from tests.gpu_util import say
from tests.test_gpu_parity import check_end_to_end

pytestmark = pytest.mark.gpu


def test_m32_edge_spaces_channelized_small():
    prob = inputs.make_problem("channel2048x1024", nx=256, ny=128, lx=0.25, ly=0.125, seed=2)
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 2, 5), label="m32 edge 256x128",
                     coef_tol=1e-8)


def test_m32_linear_spaces_all_neumann_wells():
    prob = inputs.make_problem("channel256_q5", sub=32, seed=3)
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 4, 20), label="m32 q5 256")


def test_m32_full_size_2048x1024():
    prob = inputs.make_problem("channel2048x1024", seed=1)
    g, _ = check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 2, 5), local=False,
                            label="m32 2048x1024", coef_tol=1e-8)
    st = g["stats"]
    say("  ms local %.3f interface %.3f flux %.3f (n_dof %d)"
        % (st["ms_local"], st["ms_interface"], st["ms_flux"], st["n_dof"]))


def test_m32_reduced_precision_paths_are_reported_unsupported():
    from paper_2104_04653_amd import MRCMError, MRCMSolver
    prob = inputs.make_problem("channel2048x1024", nx=128, ny=64, lx=0.125, ly=0.0625)
    for precision in ("fp32_ir", "surrogate"):
        with pytest.raises(MRCMError) as e:
            MRCMSolver(prob, precision=precision)
        assert e.value.code == 7    # MRCM_E_UNSUPPORTED
