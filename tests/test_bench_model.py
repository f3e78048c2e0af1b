"""Host logic of bench.py: the per-kernel algorithmic byte model of the
two-pass step. Record sizes, per triangle of the stage-1 pass: three corner
ids and three slot positions (4 bytes each), three parts, two kept N parts
and the kept residual (four reals each), and one CFL term per corner stored
in the triangle algebra's precision (float in the FP32 passes)."""
import bench


def test_stage1_triangle_bytes_per_triangle():
    for fp32, q in ((True, 4), (False, 8)):
        k = bench.algorithmic_bytes(1, 0, fp32)
        assert k["tri1"] == 12 + 12 + 3 * 4 * q + 2 * 4 * q + 4 * q + 3 * q
        # the CFL vertex pass reads the same per-corner terms
        assert k["cfl"] == 3 * q


def test_vertex_terms_and_precision_split():
    # per vertex: coordinates (16), Z (four reals), |v| + c (8) read by stage 1
    for fp32, q in ((True, 4), (False, 8)):
        k = bench.algorithmic_bytes(0, 1, fp32)
        assert k["tri1"] == 16 + 4 * q + 8
        assert k["cfl"] == 12
    # the FP64 model is never smaller than the FP32 one, kernel by kernel
    a, b = bench.algorithmic_bytes(1000, 500, True), bench.algorithmic_bytes(1000, 500, False)
    assert all(b[n] >= a[n] for n in a)
