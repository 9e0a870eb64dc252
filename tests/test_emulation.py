"""The library's kernel bodies run serially on the host (the FDE_EMULATE
build) and match the oracle: indexing, FFT plans and arithmetic are checked
without a GPU. The GPU tests repeat these cases on the MI355X."""
import pytest

import fde_synth
from paper_1406_7803_amd import fde

import parity_cases as pc

PRECS = [fde.F64, fde.F32]


@pytest.fixture(scope="module")
def be():
    return fde.emulation_backend()


@pytest.mark.parametrize("prec", PRECS)
def test_plan_sets(be, prec):
    pc.check_plan_sets(be, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_apply_h(be, prec):
    pc.check_apply_h(be, prec)
    pc.check_apply_h(be, prec, nb=3, with_kb=False)


@pytest.mark.parametrize("prec", PRECS)
def test_apply_h_many_projectors(be, prec):
    pc.check_apply_h_many_projectors(be, prec)
    # more than 512 bands: the projector add's vector-unit path
    pc.check_apply_h_many_projectors(be, prec, nb=520)


@pytest.mark.parametrize("prec", PRECS)
def test_density(be, prec):
    pc.check_density(be, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kin", [fde.KIN_LC94, fde.KIN_TF, fde.KIN_NONE])
def test_embed(be, prec, kin):
    pc.check_embed(be, prec, kin)


def test_embed_single_subsystem(be):
    pc.check_embed(be, fde.F64, ns=1)


@pytest.mark.parametrize("prec", PRECS)
def test_local_potential(be, prec):
    pc.check_local_potential(be, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("drop", [False, True])
def test_subspace_rr(be, prec, drop):
    pc.check_subspace_rr(be, prec, drop)


@pytest.mark.parametrize("prec", PRECS)
def test_subspace_rr_large_m(be, prec):
    pc.check_subspace_rr(be, prec, nb=45, case=pc.MEDIUM)
    pc.check_subspace_rr(be, prec, drop_case=True, nb=40, case=pc.MEDIUM)
    # m = 200, 100 bands: rotation on the matrix cores with C in chunks
    pc.check_subspace_rr(be, prec, nb=100, case=pc.MEDIUM)
    # m = 280 > 256: back-transformation with twelve rows per lane
    pc.check_subspace_rr(be, prec, nb=140, case=pc.MEDIUM)
    pc.check_subspace_rr(be, prec, drop_case=True, nb=140, case=pc.MEDIUM)


@pytest.mark.parametrize("prec", PRECS)
def test_subspace_rr_split_eigensolver(be, prec):
    """The multi-workgroup eigensolver forced on small m, alone and in a batch of mixed m."""
    pc.check_subspace_rr(be, prec, nb=45, case=pc.MEDIUM, split=1)
    pc.check_subspace_rr(be, prec, drop_case=True, nb=40, case=pc.MEDIUM, split=64)
    pc.check_subspace_rr(be, prec, nb=4, split=1)
    pc.check_subspace_rr_batched_split(be, prec, split=1)
    # and kept off for m = 280, which then takes the single-workgroup solver
    pc.check_subspace_rr(be, prec, nb=140, case=pc.MEDIUM, split=1024)


@pytest.mark.parametrize("prec", PRECS)
def test_subspace_rr_clustered_spectrum(be, prec):
    """A 40-vector eigenvalue cluster with a degenerate pair: the eigenvector phase's parallel
    iteration and workgroup orthonormalisation, in the global solver (m = 120), the split one
    (m = 120 forced, m = 300) and the LDS solver (m = 80)."""
    pc.check_subspace_rr_clustered(be, prec, 120, 60)
    pc.check_subspace_rr_clustered(be, prec, 120, 60, split=1)
    pc.check_subspace_rr_clustered(be, prec, 300, 100, case=pc.LARGE)
    pc.check_subspace_rr_clustered(be, prec, 80, 60)


def test_singular_gram(be):
    pc.check_singular_gram(be, fde.F64)


@pytest.mark.parametrize("prec", PRECS)
def test_precondition(be, prec):
    pc.check_precondition(be, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_precondition_batched(be, prec):
    pc.check_precondition_batched(be, prec)


def test_occupations(be):
    pc.check_occupations(be)


def test_trajectory_c1_fp64(be):
    pc.check_trajectory(be, fde.F64, fde_synth.config1(), 3, 1e-10, 1e-10)


def test_trajectory_kpoints_projectors(be):
    s = fde_synth.tiny(0, with_kb=True, kfrac=[(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)], grid=(12, 12, 15))
    pc.check_trajectory(be, fde.F64, s, 3, 1e-10, 1e-10)
    pc.check_trajectory(be, fde.F32, s, 3, 1e-6, 1e-5)


@pytest.mark.parametrize("grid", [(60, 48, 240), (144, 24, 432), (72, 96, 120), (180, 24, 45)])
def test_apply_h_specialised_lengths(be, grid):
    pc.check_apply_h_grid(be, fde.F64, grid)


def test_apply_h_register_z432_fp32(be):
    """432-point sticks in FP32 take the 16 x 27 register z-passes."""
    pc.check_apply_h_grid(be, fde.F32, (144, 24, 432))


def test_apply_h_register_plane(be):
    """24 x 24 planes take the register plane pass (FP64 too); three bands."""
    pc.check_apply_h_grid(be, fde.F64, (24, 24, 30), nb=3)


def test_mlp_forward(be):
    pc.check_mlp_forward(be)


def test_mlp_loss_grad(be):
    pc.check_mlp_loss_grad(be)


def test_mlp_adam(be):
    pc.check_mlp_adam(be)


@pytest.mark.parametrize("prec", PRECS)
def test_precondition_mlp(be, prec):
    pc.check_precondition_mlp(be, prec)


def test_mlp_training_reduces_loss(be):
    pc.check_mlp_training_reduces_loss(be)


def test_engine_mlp_zero_output_is_tpa(be):
    pc.check_engine_mlp_zero_output_is_tpa(be)


@pytest.mark.parametrize("gemm", [fde.GEMM_BF16X3, fde.GEMM_BF16X6])
def test_subspace_rr_bf16_split(be, gemm):
    pc.check_subspace_rr(be, fde.F32, gemm=gemm)
    pc.check_subspace_rr(be, fde.F32, drop_case=True, gemm=gemm)
    pc.check_subspace_rr(be, fde.F32, nb=40, case=pc.MEDIUM, gemm=gemm)


def test_gemm_mode_needs_fp32_plan(be):
    plan = pc.small_plan(be, fde.F64)
    with pytest.raises(fde.FdeError):
        plan.set_gemm_mode(fde.GEMM_BF16X3)


@pytest.mark.parametrize("prec", PRECS)
def test_tuning_keeps_results(be, prec):
    pc.check_tuning_keeps_results(be, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_band_energies(be, prec):
    pc.check_band_energies(be, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_grid_dot(be, prec):
    pc.check_grid_dot(be, prec)


def test_energies_c1(be):
    pc.check_energies(be, fde.F64, fde_synth.config1(), 2, 1e-10)


def test_embed_vacuum_and_empty_subsystem(be):
    pc.check_embed_grid(be, fde.F64, (24, 48, 60), 0.25)


@pytest.mark.parametrize("q0", [0.0, 0.7])
def test_mix_pulay(be, q0):
    pc.check_mix_pulay(be, fde.F64, q0)


def test_trajectory_pulay_mp(be):
    s = fde_synth.tiny(0, with_kb=True, kfrac=[(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)], grid=(12, 12, 15))
    for sub in s.subsystems:
        sub.smearing = "methfessel-paxton"
    pc.check_trajectory_pulay(be, fde.F64, s, 3, 1e-10, 1e-10, dict(kind="pulay", nhist=4, beta=0.5, q0=0.6))


@pytest.mark.parametrize("xc,xc_nad,kin", [(fde.XC_PBE, fde.XC_PBE, fde.KIN_REVAPBEK),
                                           (fde.XC_LDA, fde.XC_PBE, fde.KIN_LC94),
                                           (fde.XC_PBE, fde.XC_LDA, fde.KIN_TF),
                                           (fde.XC_PBE, fde.XC_NONE, fde.KIN_NONE)])
def test_embed_gga(be, xc, xc_nad, kin):
    pc.check_embed(be, fde.F64, kin, xc=xc, xc_nad=xc_nad)


def test_embed_gga_vacuum(be):
    pc.check_embed_grid(be, fde.F64, (24, 48, 60), 0.25, kin=fde.KIN_REVAPBEK, xc=fde.XC_PBE, xc_nad=fde.XC_PBE)


def test_trajectory_gga(be):
    pc.check_trajectory_gga(be, fde.F64, 2, 1e-10, 1e-10)


def test_supersystem_comparison(be):
    pc.check_supersystem_comparison(be, fde.F64, dict(xc=fde.XC_PBE, xc_nad=fde.XC_PBE, kin_nad=fde.KIN_LC94),
                                    n_cycles=3)


@pytest.mark.parametrize("prec", PRECS)
def test_frozen_environment(be, prec):
    pc.check_frozen_environment(be, prec)


def test_trajectory_freeze_thaw(be):
    pc.check_trajectory_freeze_thaw(be, fde.F64, 2, 2, 1e-10, 1e-10)


@pytest.mark.parametrize("prec", PRECS)
def test_augmentation(be, prec):
    pc.check_apply_s(be, prec)
    pc.check_apply_s(be, prec, nb=5, natoms=20)
    pc.check_subspace_rr_gen(be, prec)
    pc.check_aug_density(be, prec)


def test_generalised_davidson(be):
    pc.check_davidson_gen(be, fde.F64)


def test_trajectory_augmented(be):
    pc.check_trajectory_aug(be, fde.F64, 3, 1e-10, 1e-10)
