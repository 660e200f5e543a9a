"""The work model behind bench.py's rooflines, checked against closed forms
written out independently: the sparse levels' algorithmic bytes per value
size, and the flops of a dense no-pivot LU of order m."""

import bench


def counts(n=1000, m=64):
    return {"n": n, "tail_m": m, "level_nl": 7000, "level_nu": 5000, "level_macs": 110000,
            "tail_macs": 3000, "schur_macs": 2000}


def test_sparse_bytes_fp64_and_fp32():
    q = counts()
    t = q["n"] - q["tail_m"]
    # FP64: pivot 8 B; L entry 4 B index + 8 B read + 8 B write; U entry 8 B value + 8 B position;
    # multiply-add 8 B read + 8 B write + 4 B row index
    assert bench.work_model(q, 8)["sparse_bytes"] == 8 * t + 20 * 7000 + 16 * 5000 + 20 * 110000
    # FP32 values: 4 B wherever a value moves, indices and positions unchanged
    assert bench.work_model(q, 4)["sparse_bytes"] == 4 * t + 12 * 7000 + 12 * 5000 + 12 * 110000
    assert bench.work_model(q)["sparse_bytes"] == bench.work_model(q, 8)["sparse_bytes"]


def test_dense_lu_flops_closed_form():
    for m in (0, 1, 2, 64, 575):
        q = counts(n=max(m, 1) + 10, m=m)
        # step k: m-k-1 divisions and (m-k-1)^2 multiply-adds (2 flops each);
        # sum_{i<m} i + 2 i^2 = m(m-1)/2 + (m-1)m(2m-1)/3
        closed = m * (m - 1) // 2 + (m - 1) * m * (2 * m - 1) // 3 if m else 0
        assert bench.work_model(q)["dense_exec_flops"] == closed
    # leading term 2/3 m^3
    m = 34816
    q = counts(n=m + 1, m=m)
    assert abs(bench.work_model(q)["dense_exec_flops"] / (2 * m ** 3 / 3) - 1) < 1e-4
