"""Host logic of the HBM-traffic table (no GPU): counter CSVs of two
rocprofv3 runs -> bytes per launch per kernel class, scaled by the
calibration copy, keyed to the kernel source hash."""
import csv
import json

from paper_1701_02005_amd import pmc_traffic as T

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for n, (name, val) in enumerate(rows):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": n, "Kernel_Name": name, "Counter_Name": counter,
                                                 "Counter_Value": val})


def test_traffic_scaling_and_classes(tmp_path):
    copy_mb = 1024
    # the copy reads 1 GiB: FETCH_SIZE reports half of it, WRITE_SIZE all of it (KiB)
    fetch = [("__amd_rocclr_copyBuffer", copy_mb * 1024 / 2), ("__amd_rocclr_copyBuffer", 1.0),
             ("void nspnp::(anonymous namespace)::k_explicit<double, 2, 2>(nspnp::(anonymous namespace)::ExplicitArgs)", 100.0),
             ("void nspnp::(anonymous namespace)::k_explicit<double, 2, 2>(nspnp::(anonymous namespace)::ExplicitArgs)", 300.0),
             ("nspnp::(anonymous namespace)::k_cn_coef(nspnp::Dims)", 1.0),
             ("void nspnp::(anonymous namespace)::k_cn_scan<double, 3>(nspnp::(anonymous namespace)::CnArgs)", 50.0)]
    write = [("__amd_rocclr_copyBuffer", copy_mb * 1024), ("__amd_rocclr_copyBuffer", 2.0),
             ("void nspnp::(anonymous namespace)::k_explicit<double, 2, 2>(nspnp::(anonymous namespace)::ExplicitArgs)", 10.0),
             ("void nspnp::(anonymous namespace)::k_explicit<double, 2, 2>(nspnp::(anonymous namespace)::ExplicitArgs)", 30.0),
             ("nspnp::(anonymous namespace)::k_cn_coef(nspnp::Dims)", 0.0),
             ("void nspnp::(anonymous namespace)::k_cn_scan<double, 3>(nspnp::(anonymous namespace)::CnArgs)", 5.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    write_csv(fp, "FETCH_SIZE", fetch)
    write_csv(wp, "WRITE_SIZE", write)
    per, ff, fw = T.traffic(fp, wp, copy_mb)
    assert abs(ff - 2.0) < 1e-12 and abs(fw - 1.0) < 1e-12
    # k_explicit: mean 200 KiB fetched x 2, 20 KiB written
    fb, wb, n = per["k_explicit"]
    assert n == 2 and abs(fb - 200 * 2 * 1024) < 1e-6 and abs(wb - 20 * 1024) < 1e-6
    T.main(["--fetch", str(fp), "--write", str(wp), "--copy-mb", str(copy_mb), "--out", str(out)])
    tab = json.loads(out.read_text())
    ent = tab["couette_turbulent/fp64/explicit_rhs"]
    assert abs(ent["bytes_per_launch"] - (400 + 20) * 1024) < 1e-6
    assert ent["source_sha256"] == T.source_hash("stencil.hip")
    # a class is the sum of its kernels: k_cn_coef + k_cn_scan
    cn = tab["couette_turbulent/fp64/cn_tridiag"]
    assert abs(cn["bytes_per_launch"] - ((1 + 50) * 2 + 5) * 1024) < 1e-6
    # classes whose kernels were not in the runs are left out
    assert "couette_turbulent/fp64/fft_z_fwd" not in tab


def test_kernel_key():
    assert T.kernel_key("void nspnp::(anonymous namespace)::k_fft_x_r2c<double>(nspnp::Dims, ...)") == "k_fft_x_r2c"
    assert T.kernel_key("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_row_slab_cn_class(tmp_path):
    """Counter runs of the row-slab Crank-Nicolson method give the cn_tridiag
    class the sum of its two passes (and the coefficient kernel; the first pass
    runs inside the explicit kernel), and the
    entry names those kernels, so that a lane-scan figure is never reported
    for a row-slab run or the reverse."""
    copy_mb = 64
    ns = "void nspnp::(anonymous namespace)::"
    fetch = [("__amd_rocclr_copyBuffer", copy_mb * 1024 / 2), ("nspnp::(anonymous namespace)::k_cn_coef(x)", 2.0),
             (ns + "k_cn_slab_scan(x)", 3.0), (ns + "k_cn_slab_apply<float, 32>(x)", 20.0)]
    write = [("__amd_rocclr_copyBuffer", copy_mb * 1024), ("nspnp::(anonymous namespace)::k_cn_coef(x)", 0.0),
             (ns + "k_cn_slab_scan(x)", 2.0), (ns + "k_cn_slab_apply<float, 32>(x)", 4.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    write_csv(fp, "FETCH_SIZE", fetch)
    write_csv(wp, "WRITE_SIZE", write)
    T.main(["--fetch", str(fp), "--write", str(wp), "--copy-mb", str(copy_mb), "--out", str(out),
            "--workload", "couette_large", "--precision", "mixed"])
    cn = json.loads(out.read_text())["couette_large/mixed/cn_tridiag"]
    assert tuple(cn["kernels"]) == T.class_kernels("cn_tridiag", cn_slab=True)
    assert abs(cn["bytes_per_launch"] - ((2 + 3 + 20) * 2 + 2 + 4) * 1024) < 1e-6
    assert T.class_kernels("cn_tridiag", cn_slab=False) == ("k_cn_coef", "k_cn_scan")
    assert T.class_kernels("explicit_rhs", cn_slab=True) == ("k_explicit",)
