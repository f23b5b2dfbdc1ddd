"""The profile summariser's host logic: kernel names map to the kinds the
library's own profiler reports, and the shader-counter fractions follow
their stated formulas (synthetic rocprofv3 CSV rows; no GPU)."""
import csv
import os

import pytest

from paper_2511_21198_amd import rocprof_summary as rs


def _rows(names):
    return [{"Kernel_Name": n} for n in names]


def test_classify_matvec_and_preconditioner_passes():
    names = [
        "void fsd::k2_toep_x<float, 512, 0>(fsd::ToepArgs<float>)",
        "void fsd::(anonymous namespace)::k_col_toep<float, 0>(fsd::ToepArgs<float>)",
        "void fsd::(anonymous namespace)::k_col_toep<float, 1>(fsd::ToepArgs<float>)",
        "void fsd::k2_dst_x<float, 512>(fsd::DstArgs<float>)",
        "void fsd::(anonymous namespace)::k_col_dst<false>(fsd::DstArgs<float>)",
        "void fsd::(anonymous namespace)::k_col_dsth<true>(fsd::DstArgs<float>)",
        "void fsd::(anonymous namespace)::k_col_dsth<false>(fsd::DstArgs<float>)",
        "void fsd::k2_dst_s<double, 512, true>(fsd::DstArgs<double>)",
        "void fsd::k2_dst_s<double, 512, false>(fsd::DstArgs<double>)",
        "void fsd::k2_dst_s<float, 256, true, 1>(fsd::DstArgs<float>)",
        "void fsd::k2_dst_s<float, 256, false, 1>(fsd::DstArgs<float>)",
        "void fsd::k_dst_s<float, 512, 1>(fsd::DstArgs<float>)",
        "void fsd::k_dsts_s<float, 512, 1>(fsd::DstArgs<float>)",
        "void fsd::k_dstsh_s<double, 512, 8>(fsd::DstArgs<double>)",
        "void fsd::k2_toep_x<float, 512, 3, 2>(fsd::ToepArgs<float>)",
        "void fsd::k_mdot<float, 4>(fsd::MdotArgs)",
        "some_other_kernel",
    ]
    assert rs.classify(_rows(names)) == [
        "toep_x_f32", "toep_y_f32", "toep_z_f32", "dst_x_f32", "dst_y_f32", "dsts_z_f32",
        "dst_y_f32", "dsts_z_f64", "dst_y_f64", "dsts_z_f32", "dst_y_f32", "dst_y_f32",
        "dsts_z_f32", "dsts_z_f64", "toep_x_f32", "gm_mdot_f32", None]


def test_sq_summary_fractions(tmp_path):
    d = tmp_path / "sq" / "host"
    os.makedirs(d)
    rows = []
    vals = {"SQ_WAVES": 1000, "SQ_INSTS_VALU": 500000, "SQ_INSTS_LDS": 100000,
            "SQ_ACTIVE_INST_VALU": 256000, "SQ_ACTIVE_INST_LDS": 128000,
            "SQ_LDS_BANK_CONFLICT": 25600, "SQ_BUSY_CYCLES": 2000, "SQ_WAVE_CYCLES": 9000,
            "GRBM_GUI_ACTIVE": 1000}
    for disp, scale in ((1, 1.0), (2, 0.01)):     # the second returned at once
        for c, v in vals.items():
            rows.append({"Dispatch_Id": disp, "Kernel_Name": "void fsd::k2_dst_x<float, 512>(x)",
                         "Counter_Name": c, "Counter_Value": v * (scale if c == "SQ_INSTS_VALU" else 1)})
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    out = rs.sq_summary(str(tmp_path / "sq"))
    e = out["dst_x_f32"]
    assert e["dispatches"] == 1
    c = 1000 / 8      # busy cycles: the GRBM counter sums the 8 dies
    assert e["valu_busy"] == pytest.approx(4 * 256000 / (1024 * c))
    assert e["lds_busy"] == pytest.approx(4 * 128000 / (1024 * c))
    assert e["bank_conflict"] == pytest.approx(25600 / (256 * c))
    assert e["valu_per_wave"] == pytest.approx(500.0)
