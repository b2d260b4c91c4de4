"""Sanitizer runs of the CPU oracle and of the library's host-only code (no GPU).

The oracle (oracle/oracle.c) is built with AddressSanitizer and
UndefinedBehaviorSanitizer into a small driver (tests/sanitize/oracle_main.c)
and run on designs that reach every operation type, fused mux chains,
multi-limb registers of 64 to 256 bits and a design without registers; any
out-of-bounds access, leak, signed overflow, shift past the width or other
undefined behaviour aborts the driver.  Its results must also equal the
normal build's.  The library's host code (include/rteaal.h validation and
mux-chain fusion, which touch no GPU) is built the same way
(tests/sanitize/host_main.c) and must agree with the unsanitized library.
The whole host runtime (batches, multi-batch steps and their captured-cycle
cache, read-out, autotuners) runs the call sequences of
tests/sanitize/host_scenarios.cpp against a host-only stand-in for the HIP
runtime (tests/sanitize/hip_mock.cpp) that also checks every launch's
memory, at launch and at every later replay of a captured graph.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
import rtlgen
from rtlgen import circuits as cir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def write_design(path, d, seeds, cycles, threads=2):
    seeds = np.asarray(seeds, np.uint64)
    with open(path, "wb") as f:
        f.write(struct.pack("<10I2Q", 0x524F5452, d.n_slots, d.const_slot.size, d.input_slot.size,
                            d.reg_slot.size, d.layer_ptr.size - 1, d.op_type.size,
                            int(d.op_src_ptr[-1]), seeds.size, threads, 0, cycles))
        for a, dt in ((d.slot_width, np.uint16), (d.const_slot, np.uint32),
                      (np.asarray(d.const_limbs).reshape(-1), np.uint64), (d.input_slot, np.uint32),
                      (d.reg_slot, np.uint32), (d.reg_next, np.uint32), (d.layer_ptr, np.uint32),
                      (d.op_type, np.uint8), (d.op_dst, np.uint32), (d.op_src_ptr, np.uint32),
                      (d.op_src, np.uint32), (d.op_imm, np.uint16), (seeds, np.uint64)):
            f.write(np.ascontiguousarray(a, dtype=dt).tobytes())


def designs():
    out = [("all-types", rtlgen.generate(rtlgen.GenConfig(
        400, 8, 24, 8, rtlgen.generator.WIDTHS_LARGE, "san-all", rtlgen.OP_MIX_FULL), 3)),
        ("wide", rtlgen.generate(rtlgen.GenConfig(600, 9, 40, 10, rtlgen.generator.WIDTHS_LARGE,
                                                  "san-wide"), 4)),
        ("no-regs", rtlgen.generate(rtlgen.GenConfig(200, 4, 0, 6, rtlgen.generator.WIDTHS_STD,
                                                     "san-noregs"), 5))]
    chains = rtlgen.generate(rtlgen.GenConfig(800, 10, 32, 8, rtlgen.generator.WIDTHS_STD,
                                              "san-chains", mux_chain=0.85), 6)
    fused, n_fused, _ = oracle.fuse_mux_chains(chains)
    assert n_fused > 0
    out += [("chains", chains), ("fused", fused)]
    out += [(f"counter{w}", cir.counter(w, 3**(w // 2) + 1)) for w in (64, 65, 128, 200, 256)]
    return out


@pytest.fixture(scope="module")
def oracle_asan(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("no clang with sanitizer runtimes")
    exe = str(tmp_path_factory.mktemp("san") / "oracle_asan")
    subprocess.run([CLANG, *SAN_FLAGS, "-std=c11", "-pthread", os.path.join(SAN, "oracle_main.c"),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("name,d", designs(), ids=[n for n, _ in designs()])
def test_oracle_under_sanitizers(oracle_asan, tmp_path, name, d):
    seeds = [1, 77, 2**63 + 5]
    cyc = 30
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_design(inp, d, seeds, cyc)
    r = subprocess.run([oracle_asan, inp, out], env=ENV, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    raw = np.fromfile(out, dtype=np.uint64)
    n_reg_words = len(seeds) * d.n_regs * 4
    dg = {}
    ref, _, _ = oracle.run(d, seeds, cyc, digests=dg)
    assert np.array_equal(raw[:n_reg_words].reshape(ref.shape), ref)
    assert np.array_equal(raw[n_reg_words:], dg["final"])


@pytest.fixture(scope="module")
def host_asan(tmp_path_factory):
    """The library's host code (host.cpp) built with host-side sanitizers
    (device code unchanged), linked with the library's kernel objects."""
    if not (os.path.exists(CLANG) and shutil.which("hipcc")):
        pytest.skip("no hipcc / clang with sanitizer runtimes")
    from paper_2601_18140_amd import build as B
    objdir = os.path.join(ROOT, "paper_2601_18140_amd", "_build")
    objs = [os.path.join(objdir, f) for f in ("kernels.hip.o", "levelize.hip.o")]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    tmp = tmp_path_factory.mktemp("hsan")
    host_o, main_o, exe = str(tmp / "host.o"), str(tmp / "main.o"), str(tmp / "host_asan")
    host_flags = [f for f in SAN_FLAGS if f.startswith("-f")]
    cmd = ["hipcc", "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    for f in host_flags:
        cmd += ["-Xarch_host", f]
    subprocess.run(cmd + ["-c", os.path.join(ROOT, "paper_2601_18140_amd", "csrc", "host.cpp"),
                          "-o", host_o], check=True, capture_output=True)
    subprocess.run([CLANG, *SAN_FLAGS, "-c", os.path.join(SAN, "host_main.c"), "-o", main_o],
                   check=True)
    subprocess.run([CLANG + "++", "-fsanitize=address,undefined", main_o, host_o, *objs,
                    "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                   check=True)
    return exe


@pytest.mark.parametrize("max_pairs", [32, 2])
@pytest.mark.parametrize("name,d", designs(), ids=[n for n, _ in designs()])
def test_host_validate_and_fuse_under_sanitizers(host_asan, tmp_path, name, d, max_pairs):
    from paper_2601_18140_amd import rteaal as R
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_design(inp, d, [1], 1)
    # The HIP runtime's own allocations at start-up are not this code's:
    # leaks are not checked here (the oracle test above checks them).
    env = dict(ENV, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0")
    r = subprocess.run([host_asan, inp, out, str(max_pairs)], env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    raw = open(out, "rb").read()
    vs = struct.unpack_from("<i", raw, 0)[0]
    assert vs == R.rteaal_validate_design(d)[0] == 0
    fs, n_ops, n_operands, n_fused, n_absorbed = struct.unpack_from("<i4I", raw, 4)
    assert fs == 0
    exp, cnt = R.rteaal_fuse_mux_chains(d, max_pairs)
    assert (n_ops, n_operands, n_fused, n_absorbed) == (cnt["n_ops"], cnt["n_operands"],
                                                        cnt["n_fused"], cnt["n_absorbed"])
    off = 24
    nl = d.layer_ptr.size
    for name_, dt, n in (("layer_ptr", np.uint32, nl), ("op_type", np.uint8, n_ops),
                         ("op_dst", np.uint32, n_ops), ("op_src_ptr", np.uint32, n_ops + 1),
                         ("op_src", np.uint32, n_operands), ("op_imm", np.uint16, n_ops)):
        a = np.frombuffer(raw, dtype=dt, count=n, offset=off)
        off += a.nbytes
        assert np.array_equal(a, np.asarray(getattr(exp, name_))), name_


@pytest.fixture(scope="module")
def host_scenarios(tmp_path_factory):
    """The library's host code with a host-only stand-in for the HIP runtime
    and the kernel launchers (tests/sanitize/hip_mock.cpp), and the call
    sequences of tests/sanitize/host_scenarios.cpp, all under ASan and
    UBSan."""
    if not (os.path.exists(CLANG) and shutil.which("hipcc")):
        pytest.skip("no hipcc / clang with sanitizer runtimes")
    from paper_2601_18140_amd import build as B
    tmp = tmp_path_factory.mktemp("scen")
    host_o, mock_o, scen_o, exe = (str(tmp / f) for f in ("host.o", "mock.o", "scen.o", "scen"))
    cmd = ["hipcc", "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    for f in SAN_FLAGS:
        if f.startswith("-f"):
            cmd += ["-Xarch_host", f]
    subprocess.run(cmd + ["-c", os.path.join(ROOT, "paper_2601_18140_amd", "csrc", "host.cpp"),
                          "-o", host_o], check=True, capture_output=True)
    subprocess.run([CLANG + "++", *SAN_FLAGS, "-std=c++17", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-c", os.path.join(SAN, "hip_mock.cpp"), "-o", mock_o],
                   check=True)
    subprocess.run([CLANG + "++", *SAN_FLAGS, "-std=c++17", "-c",
                    os.path.join(SAN, "host_scenarios.cpp"), "-o", scen_o], check=True)
    subprocess.run([CLANG + "++", "-fsanitize=address,undefined", scen_o, mock_o, host_o, "-o", exe],
                   check=True)
    return exe


def test_host_runtime_scenarios_under_sanitizers(host_scenarios, tmp_path):
    """Batches of every mapping through rteaal_step_many (uneven cycle counts,
    a batch of a cached set freed, more sets than the cache holds, stimulus
    words, watched and timed batches), read-out and restore, and both
    autotuners: no sanitizer report, no leak, no launch on freed memory."""
    files = []
    for k, c in enumerate([rtlgen.GenConfig(700, 6, 30, 8, rtlgen.generator.WIDTHS_LARGE, "sc-a"),
                           rtlgen.GenConfig(1300, 17, 50, 12, rtlgen.generator.WIDTHS_MULTIDESIGN,
                                            "sc-b"),
                           rtlgen.GenConfig(400, 3, 20, 6, rtlgen.generator.WIDTHS_STD, "sc-c")]):
        f = str(tmp_path / f"d{k}.bin")
        write_design(f, rtlgen.generate(c, 50 + k), [1], 1)
        files.append(f)
    r = subprocess.run([host_scenarios, *files], env=ENV, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "scenarios ok" in r.stdout
