"""The formulation options of the interaction on the GPU against the CPU
oracle, through the C ABI: the cubic spline kernel (Eq. 10), laminar
viscosity (Eq. 23), the Fourtakas density diffusion (Eq. 19-20) and all three
together.  Same bars as the default formulation: FP64-test neighbour counts
bit-exact, rates within 1e-4 of max|oracle|, FP32 count flips only at
near-ties."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2104_00537_amd import cases

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from test_gpu_parity import _check_interact, _perturbed

VARIANTS = {
    "cubic": dict(kernel=1),
    "laminar": dict(viscosity=1, visc_nu=1e-2),
    "fourtakas": dict(ddt=2),
    "all": dict(kernel=1, viscosity=1, visc_nu=1e-2, ddt=2),
}


def _variant(case, **kw):
    return cases.Case(dataclasses.replace(case.params, **kw), case.pos, case.vel, case.rho,
                      case.type, dict(case.meta))


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_2d_dam_break(name):
    c = _perturbed(cases.dam_break_2d(cell_div=2, x_sub=4), 31, vel=0.5)
    _check_interact(_variant(c, **VARIANTS[name]), f"2d {name}")


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_3d_block_with_walls(name):
    c = cases.block_case(3, (21, 17, 15), walls=True, seed=7, cell_div=2, x_sub=4)
    _check_interact(_perturbed(_variant(c, **VARIANTS[name]), 32, vel=0.3), f"3d {name}")
