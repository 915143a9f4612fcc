"""The reverse-Poiseuille viscometer (Sec. 4.1) and the slurry experiment
(Sec. 4.3) end to end on the GPU at the paper's fluid constants (eta = 25,
rho0 = 3, p0 = beta = 100, drive 1.5): the fully periodic channel's
viscosity, the wall-periodic channel against it, and the slurry's viscosity
rising with concentration.  Every step runs in the HIP library; the host
only bins velocities and fits the profiles."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def result():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import slurry
    print("[case] slurry experiment: 2 channels + 3 concentrations, 3500 steps each", flush=True)
    return slurry.experiment(log=lambda m: print(m, flush=True))


def test_periodic_channel_viscosity(result):
    """The SDPD fluid's measured viscosity sits below its input eta (at
    h = 2 dx and kT = 1 the disordered particles transmit about 0.88 eta);
    the periodic images put the no-slip planes on the box faces."""
    r = result
    assert 0.8 * r["eta"] < r["mu_periodic"] < 1.0 * r["eta"]
    assert abs(r["periodic_slip_delta"]) < 0.1
    assert r["se_mu_periodic"] < 0.01 * r["mu_periodic"]


def test_wall_periodic_channel_matches_periodic(result):
    """With walls on the z faces the no-slip plane lies about one spacing
    outside the face (the inner wall layer moves like fluid); with that
    plane fitted the two boundary conditions give viscosities within 2 %,
    the agreement the paper reports."""
    r = result
    assert abs(r["rel_diff_wall_vs_periodic_fitted_plane"]) < 0.02
    assert 0.25 < r["wall_slip_delta"] < 0.75
    # read with the planes on the faces (Eq. poiseuave as printed) the slip
    # shows as a lower viscosity
    assert r["mu_wall_periodic"] < r["mu_periodic"]


def test_slurry_viscosity_rises_with_concentration(result):
    sl = result["slurry"]
    assert [round(100 * s["concentration"], 2) for s in sl] == [3.67, 5.5, 11.0]
    prev_mu, prev_se = result["mu_wall_periodic"], result["se_mu_wall_periodic"]
    for s in sl:
        assert s["mu"] - prev_mu > 3.0 * (s["se_mu"] ** 2 + prev_se ** 2) ** 0.5
        prev_mu, prev_se = s["mu"], s["se_mu"]
    assert sl[0]["relative_viscosity"] > 1.0
