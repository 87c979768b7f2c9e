"""Magnetically driven sphere on the GPU (through the C ABI): the same case as
test_magnetic_sphere.py, FP64 plain and FP32 mixed, against the oracle and the
growth law dR/dn = beta b - kappa_s sigma^2 / R."""
import numpy as np
import pytest

import test_magnetic_sphere as ms
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _gpu(precision, energy=None):
    import paper_1701_06658_amd as gg

    def make(labels):
        if energy is None:
            return gg.Simulation(labels, ms.W, G=2, precision=precision)
        return gg.Simulation(labels, ms.W, G=2, precision=precision, physics=gg.PHYS_BULK, energy=energy,
                             voxel_m=ms.H, gamma_max=ms.GAMMA)
    return make


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gpu_magnetic_sphere(precision):
    steps, r_star = 12, 9.0
    kappa_o = ms.kappa_from_curvature(ms._run(lambda lab: Oracle(lab, ms.W, G=2), 10))
    kappa_g = ms.kappa_from_curvature(ms._run(_gpu(precision), 10))
    energy, b = ms.energies_for(r_star, kappa_o)
    ro = ms._run(lambda lab: Oracle(lab, ms.W, G=2), steps, energy)
    rg = ms._run(_gpu(precision, energy), steps)
    law = ms.law_radius(ro[0], b, kappa_o, steps)
    tol = 1e-9 if precision == "fp64" else 2e-3
    print(f"[{precision}] kappa oracle {kappa_o:.6f} gpu {kappa_g:.6f}; max |R_gpu - R_oracle| "
          f"{np.max(np.abs(rg - ro)):.3e}; max |R_gpu - law| {np.max(np.abs(rg - law)):.3e}", flush=True)
    assert abs(kappa_g - kappa_o) <= (1e-9 if precision == "fp64" else 5e-3 * kappa_o)
    assert np.max(np.abs(rg - ro)) <= tol
    change = abs(law[-1] - law[0])
    assert np.max(np.abs(rg[:4] - law[:4])) <= 0.04 * abs(law[3] - law[0]) + 0.005
    assert np.max(np.abs(rg - law)) <= 0.12 * change
