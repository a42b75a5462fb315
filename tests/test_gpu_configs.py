"""The workload-level checks of tests/config_checks.py as GPU tests: the
rotor channel over 20,000 steps, the adjoint gradient of the 128x64x64
workload against central differences, the wake profiles of the coarse
wake copy against the FP64 oracle, and FP16 against FP32 per-rotor torque
on the 1536x768x256 array."""
import os

import numpy as np
import pytest

import config_checks as CC

pytestmark = pytest.mark.gpu


def test_c2_rotor_channel_20k_steps_is_stable():
    r = CC.c2_long_run()
    print(f"[configs] c2: {r['seconds']} s, mass/cell {r['mass_per_cell_first_last']}, torque mean "
          f"{r['torque_mean_last5000']:.3f} +- {r['torque_std_last5000']:.3f}, by 4000 steps "
          f"{[round(v, 2) for v in r['torque_mean_by_4000']]}", flush=True)
    assert r["stable"] and r["finite"]
    # statistically steady after the start-up: block means within 5 %
    m = np.array(r["torque_mean_by_4000"][1:])
    assert np.abs(m - m.mean()).max() < 0.05 * abs(m.mean())


def test_c4_adjoint_against_central_differences():
    """32 seeded cells of the rotor's cylinder, J = mean axial torque over
    steps [1000, 2000).  With eps = 1e-5 no wall-model Newton stop decision
    flips and the FP64 adjoint equals the differences to their truncation
    error; with eps = 1e-3 (stated) the decisions flip on some cells and J
    jumps there, which the adjoint (iterations differentiated as executed)
    does not see."""
    r = CC.c4_gradient()
    small, big = r["eps_1e-05"], r["eps_0.001"]
    print(f"[configs] c4: eps 1e-5 max err f64 {small['max_err_f64']:.2e} f32 {small['max_err_f32']:.2e}; "
          f"eps 1e-3 max err {big['max_err_f64']:.2e} median {big['median_rel_err_f64']:.2e} corr "
          f"{big['corr_f64']:.4f}; FP32 vs FP64 adjoint {r['f32_vs_f64_adjoint']:.2e}", flush=True)
    assert small["max_err_f64"] < 1e-4
    assert small["max_err_f32"] < 2e-3
    assert r["f32_vs_f64_adjoint"] < 2e-3


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(__file__), "golden",
                                                    "wake_profiles_256x128x96.json")),
                    reason="oracle wake profiles not generated")
def test_c3_wake_profiles_against_the_oracle():
    r = CC.c3_profiles()
    for st, v in r["storages"].items():
        print(f"[configs] c3 {st}: L2 rel diff at 2R, 5R {v['l2_rel_2R_5R']}, max |diff| / U "
              f"{v['max_abs_over_U_2R_5R']}", flush=True)
    for st, v in r["storages"].items():
        assert max(v["l2_rel_2R_5R"]) < 0.05, (st, v["l2_rel_2R_5R"])


def test_c5_fp16_against_fp32_rotor_torque():
    r = CC.c5_torque()
    print(f"[configs] c5: FP16 vs FP32 mean axial torque over steps {r['window']}: rel diff per rotor "
          f"{[f'{v:.1e}' for v in r['rel_diff_per_rotor']]}", flush=True)
    assert r["rel_diff_max"] < 1e-3
