"""The bench's byte model (host only): value sizes and the algorithmic bytes
of one instance-cycle, checked against a small design worked by hand."""
import numpy as np

import bench
import rtlgen
from rtlgen import circuits as cir


def test_value_sizes():
    w = np.array([1, 2, 8, 9, 16, 17, 32, 33, 64, 65, 128, 129, 256])
    assert list(bench.wb(w)) == [0.125, 4, 4, 4, 4, 4, 4, 8, 8, 16, 16, 24, 32]
    assert list(bench.eb(w)) == [0.125, 1, 1, 2, 2, 4, 4, 8, 8, 16, 16, 24, 32]


def test_algorithmic_bytes_by_hand():
    b = cir.Builder("bytes")
    a, bb, s, c = b.input(8), b.input(8), b.input(1), b.input(100)
    x = b.op(rtlgen.ADD, [a, bb], 8)                     # light: 4 + 4 + 4 = 12
    p = b.op(rtlgen.ADD, [c, c], 100)                    # heavy (wide): 16 + 16 + 16 = 48
    m = b.op(rtlgen.MUXC, [s, a, s, bb, a], 8)           # heavy (type): 1/8 + 4 + 1/8 + 4 + 4 + 4
    y = b.op(rtlgen.MUX, [s, x, a], 8)                   # light: 1/8 + 4 + 4 + 4
    r1, r2 = b.reg(8), b.reg(100)
    b.connect(r1, y)                                     # commit: 4 + 4 (light)
    b.connect(r2, p)                                     # commit: 16 + 16 (heavy)
    _ = m
    d = b.build()
    ab = bench.algorithmic_bytes(d)
    assert ab["x_light"] == 12 + 12.125 + 8
    # inputs (4 + 4 + 1/8 + 16 bytes) count with the heavy kernel, which writes them
    assert ab["x_heavy"] == 48 + 16.25 + 32 + 24.125
    assert ab["x"] == ab["x_light"] + ab["x_heavy"]
    # graph bytes: per operation (1 + arity) coordinates at the layer's bit
    # width, a 9-bit type code; layer 0 holds x, p, m (largest slot index 6 ->
    # 3 bits), layer 1 holds y (index 7 -> 3 bits)
    g0 = ((1 + 2) * 3 + 9) / 8 + ((1 + 2) * 3 + 9) / 8 + ((1 + 5) * 3 + 9) / 8
    g1 = ((1 + 3) * 3 + 9) / 8
    assert abs(ab["g"] - (g0 + g1)) < 1e-9
    assert abs(ab["g_heavy"] - (((1 + 2) * 3 + 9) / 8 + ((1 + 5) * 3 + 9) / 8)) < 1e-9
    # the storage encoding moves 1 byte for each 8-bit value instead of 4
    ae = bench.algorithmic_bytes(d, bench.eb)
    assert ae["x_light"] == 3 + 3.125 + 2


def test_more_than_one_gpu_is_refused():
    """bench.py runs on one GPU; --gpus N > 1 exits with a message, before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
