"""Shell transfers and the acoustic wave on the GPU (section 3.4: solution transfer
on curved elements with the reference matrices, volume loss; section 4.4: the
acoustic wave around the globe).

dg_sphere_refine_project and dg_sphere_coarsen_project against the oracle's
refine_shell / coarsen_shell at N = 2..5 (fields, the scale factor, the total mass
kept by refinement), the volume ratio as the scale factor on a constant-density
background, and the acoustic state run for 18 hours on a coarse shell: the
pressure pulse at the antipode of the initial bell is centred on
pi r_e / c = 16.0 hours (c = 347.3 m/s, the paper's estimate and observation),
with the mass kept to round-off over the run.  The wave runs without gravity, as
the paper's two-dimensional shallow-atmosphere problem: with gravity and the
isothermal (stably stratified) background, elements a layer of 10 km tall let
the strong-form operator grow a buoyancy-coupled mode within an hour (the
oracle does the same in a box), which finer layers delay."""
import math

import numpy as np
import pytest
import torch

from oracle import euler as eu
from oracle import sphere as sp
from paper_2404_16648_amd import dg
from paper_2404_16648_amd.synth import random_state
from tests.helpers import TOL_FP64, assert_conserved_fields, assert_fields, to_elem, to_nodes
from tests.test_gpu_parity import gpu

pytestmark = pytest.mark.gpu

PH = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL)
OPH = eu.Phys()


def _pair(N, n, nz, kind=sp.BG_ISOTHERMAL, oph=OPH):
    lc, lf = dg.dg_sphere_mesh_build(N, n, nz), dg.dg_sphere_mesh_build(N, 2 * n, 2 * nz)
    oc = sp.SphereOperator(sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz)), oph, kind)
    of = sp.SphereOperator(sp.SphereMesh(sp.SphereDesc(N=N, n=2 * n, nz=2 * nz)), oph, kind)
    return lc, lf, oc, of


@pytest.mark.parametrize("N,n,nz", [(2, 1, 1), (3, 2, 1), (4, 2, 1), (5, 1, 1)])
def test_shell_transfers_against_oracle(N, n, nz):
    lc, lf, oc, of = _pair(N, n, nz)
    print(f"shell transfer N={N} n={n} nz={nz} Kc={oc.K} Kf={of.K}", flush=True)
    qn = torch.as_tensor(random_state(oc.K, N, 60 + N)) * 0.1
    qn = qn + to_nodes(sp.acoustic_state(oc))
    qf = lf.field()
    s = dg.dg_sphere_refine_project(lc, lf, PH, gpu(qn), qf)
    q_ref, s_ref = sp.refine_shell(oc, of, to_elem(qn, N))
    print("scale", s, s_ref, flush=True)
    assert abs(s - s_ref) <= 1e-15 * s_ref
    assert_fields(qf, to_nodes(q_ref), TOL_FP64, "shell refine")
    b0, b1 = dg.dg_budgets(lc, PH, gpu(qn)), dg.dg_budgets(lf, PH, qf)
    assert abs(b1[1] - b0[1]) <= 1e-15 * b0[1], (b0[1], b1[1])
    # coarsening of a state on the fine shell (the refined one plus its own noise)
    qfn = qf.cpu() + torch.as_tensor(random_state(of.K, N, 70 + N)) * 0.05
    qc = lc.field()
    dg.dg_sphere_coarsen_project(lf, lc, PH, gpu(qfn), qc)
    torch.cuda.synchronize()
    qc_ref = sp.coarsen_shell(of, oc, to_elem(qfn, N))
    assert_conserved_fields(qc, to_nodes(qc_ref), (to_nodes(oc.bg[0][None])[0], to_nodes(oc.bg[1][None])[0]), TOL_FP64,
                            "shell coarsen")


def test_scale_factor_is_the_volume_ratio():
    N, n, nz = 3, 2, 1
    ph = dg.PhysParams(background=dg.DG_BG_CONSTANT, g=0.0)
    lc, lf = dg.dg_sphere_mesh_build(N, n, nz), dg.dg_sphere_mesh_build(N, 2 * n, 2 * nz)
    s = dg.dg_sphere_refine_project(lc, lf, ph, lc.field(), lf.field())
    _, (vc, _) = dg.dg_sphere_volumes(lc)
    _, (vf, _) = dg.dg_sphere_volumes(lf)
    print("volume loss", vf / vc - 1.0, "scale", s, flush=True)
    assert abs(s - vc / vf) <= 1e-15
    assert 0.0 < vf / vc - 1.0 < 1e-3


def test_shell_transfer_refusals():
    lc, lf = dg.dg_sphere_mesh_build(3, 2, 1), dg.dg_sphere_mesh_build(3, 4, 2)
    with pytest.raises(dg.DGError) as e:
        dg.dg_sphere_refine_project(lc, lf, dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, mu=1.5),
                                    lc.field(), lf.field())
    assert e.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as e:
        dg.dg_sphere_refine_project(lf, lc, PH, lf.field(), lc.field())
    assert e.value.code == dg.DG_EINVAL


def test_acoustic_wave_reaches_the_antipode_after_16_hours():
    """Section 4.4's acoustic wave (cosine bell of 100 Pa and radius r_e/3 times
    sin(pi h / H)) on a 6 x 12 x 12 x 1 shell, N = 4, dt = 0.9 s (vertical Courant
    number 0.18), as the paper's two-dimensional shallow-atmosphere problem: no
    gravity (it acts normal to the surface the 2-D problem lives on), so the 300 K
    background is uniform.  The mean pressure perturbation over the nodes within
    300 km of the antipode, sampled every 5 minutes from 14 to 18 hours, rises to a
    positive lobe and falls to a negative one; the zero crossing between them and
    the mid-point of the two extrema lie within 1.5% of pi r_e / c; the mass changes
    by round-off only."""
    N, n, nz, dt = 4, 12, 1, 0.9
    ph = dg.PhysParams(background=dg.DG_BG_ISOTHERMAL, g=0.0)
    oph = eu.Phys(g=0.0)
    lm = dg.dg_sphere_mesh_build(N, n, nz)
    om = sp.SphereMesh(sp.SphereDesc(N=N, n=n, nz=nz))
    op = sp.SphereOperator(om, oph, sp.BG_ISOTHERMAL)
    q = gpu(to_nodes(sp.acoustic_state(op)))
    rho_b, Th_b, P_b = (to_nodes(b[None])[0] for b in op.bg)
    dist = 6.371e6 * torch.arccos(torch.clamp(-op.geo.rhat[0], -1.0, 1.0))
    sel = to_nodes(dist[None])[0] <= 3.0e5
    assert int(sel.sum()) >= 4
    idx = torch.nonzero(sel.reshape(-1)).reshape(-1)
    Thb_s, Pb_s = Th_b.reshape(-1)[idx], P_b.reshape(-1)[idx]
    idx_d = idx.cuda()
    gamma = oph.gamma

    def antipode_pressure():
        thp = q[4].reshape(-1)[idx_d].cpu()
        return float(eu.pressure_perturbation(thp, Thb_s, Pb_s, gamma).mean())

    a, b = lm.field(), lm.field()
    b0 = dg.dg_budgets(lm, ph, q)
    t, times, vals = 0.0, [], []
    t_first, t_end, every = 14.0 * 3600.0, 18.0 * 3600.0, 300.0
    nsteps = 0
    next_sample = t_first
    while t < t_end - 1e-9:
        dg.ssp_rk3_step(lm, ph, dt, q, a, b)
        t += dt
        nsteps += 1
        if t >= next_sample - 1e-9:
            times.append(t)
            vals.append(antipode_pressure())
            next_sample += every
            if len(times) % 6 == 0:
                print(f"acoustic wave: t = {t / 3600.0:.2f} h, antipode p' = {vals[-1]:.4f} Pa", flush=True)
    b1 = dg.dg_budgets(lm, ph, q)
    vals = np.array(vals)
    times = np.array(times)

    def vertex(i):
        """time of the extremum of the parabola through samples i - 1, i, i + 1"""
        assert 0 < i < len(vals) - 1, vals
        y0, y1, y2 = vals[i - 1], vals[i], vals[i + 1]
        return times[i] + 0.5 * every * (y0 - y2) / (y0 - 2.0 * y1 + y2)

    # the pulse that converges on the antipode arrives as a positive lobe followed by
    # a negative one (the two-dimensional wave's focus); its centre, where p' crosses
    # zero between the lobes, is the arrival of the bell's centre
    i_max, i_min = int(np.argmax(vals)), int(np.argmin(vals))
    assert i_max < i_min
    t_max, t_min = vertex(i_max), vertex(i_min)
    j = i_max + int(np.argmax(vals[i_max:] < 0.0))
    t_zero = times[j - 1] + every * vals[j - 1] / (vals[j - 1] - vals[j])
    c = math.sqrt(gamma * oph.R * oph.theta0)
    t_exp = math.pi * 6.371e6 / c
    print(f"antipode p': +{vals[i_max]:.2f} Pa at {t_max / 3600.0:.3f} h, {vals[i_min]:.2f} Pa at "
          f"{t_min / 3600.0:.3f} h, zero at {t_zero / 3600.0:.3f} h; pi r_e / c = {t_exp / 3600.0:.3f} h "
          f"(c = {c:.2f} m/s); {nsteps} steps; mass change {(b1[1] - b0[1]) / b0[1]:.2e}, "
          f"energy change {(b1[3] - b0[3]) / abs(b0[3]):.2e}", flush=True)
    assert abs(t_zero / t_exp - 1.0) <= 0.015
    assert abs(0.5 * (t_max + t_min) / t_exp - 1.0) <= 0.015
    assert vals[i_max] > 10.0 and 0.5 < -vals[i_min] / vals[i_max] < 2.0
    assert abs(b1[1] - b0[1]) <= 1e-13 * b0[1]
