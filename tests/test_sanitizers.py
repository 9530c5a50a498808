"""The oracle and the library's host code under the address and
undefined-behaviour sanitizers.

``oracle/sanitize_check.c`` runs every oracle entry point on a scene file
(BVH and brute-force renders of the three displacement mappings compared
bit for bit, selected chains, one pass with hit data, batched closest hits
against single queries, shading, normals and the screen-space passes in the
three edge modes).  Built with ``-fsanitize=address,undefined`` and halting on
the first report, any out-of-bounds access, use after free, leak, signed
overflow, misaligned access or bad shift in the oracle fails the test.

The library's host code (argument checks, workspaces, graphs, the server's
scheduler thread, the autotuner, error paths) is built the same way by
``build_sanitized`` (device code unchanged) and driven by
``tests/sanitize_host_check.cpp``: its argument-validation part runs here on
the CPU, and the whole driver, every entry point on the device, runs in the
GPU test below.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import scenegen
from paper_2312_12392_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

SAN_FLAGS = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-pthread",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    out = str(tmp_path_factory.mktemp("san") / "sanitize_check")
    subprocess.check_call(["gcc", *SAN_FLAGS, "-I", ORACLE, "-o", out,
                           os.path.join(ORACLE, "sanitize_check.c"), os.path.join(ORACLE, "rcp_oracle.c"), "-lm"])
    return out


def write_scene(path, scene):
    with open(path, "wb") as f:
        f.write(np.array([scene.n_verts, scene.n_tris], dtype="<u4").tobytes())
        f.write(scene.verts.astype("<f4").tobytes())
        f.write(scene.idx.astype("<u4").tobytes())
        f.write(scene.rgb.astype("<f4").tobytes())


SCENES = {
    "terrain_patch": lambda: scenegen.terrain_patch(11, cells=12, n_boxes=4),
    "adversarial": lambda: scenegen.adversarial_scene(5),
    "soup": lambda: scenegen.soup_scene(2, n=300),
    "single_quad": lambda: scenegen.quad_scene(0.2),
    "empty": scenegen.empty_scene,
}


@pytest.mark.parametrize("name", list(SCENES))
def test_oracle_clean_under_asan_ubsan(checker, tmp_path, name):
    scene = SCENES[name]()
    path = str(tmp_path / "scene.bin")
    write_scene(path, scene)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1:verify_asan_link_order=0:exitcode=99"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=98"
    r = subprocess.run([checker, path], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert "runtime error" not in report and "Sanitizer" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "ok" in r.stdout


def test_sanitizer_catches_a_planted_overrun(tmp_path):
    """The harness itself: a copy of the oracle whose screen-space pass runs
    one column past the row must be reported (and exit non-zero)."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    src = open(os.path.join(ORACLE, "rcp_oracle.c")).read()
    at = src.index("int orc_gather_pass(")
    loop = "for (int x = 0; x < W; ++x) {"
    j = src.index(loop, at)
    bad = src[:j] + "for (int x = 0; x <= W; ++x) {" + src[j + len(loop):]
    (tmp_path / "rcp_oracle.c").write_text(bad)
    shutil.copy(os.path.join(ORACLE, "rcp_oracle.h"), tmp_path / "rcp_oracle.h")
    exe = str(tmp_path / "planted")
    subprocess.check_call(["gcc", *SAN_FLAGS, "-I", str(tmp_path), "-o", exe,
                           os.path.join(ORACLE, "sanitize_check.c"), str(tmp_path / "rcp_oracle.c"), "-lm"])
    path = str(tmp_path / "scene.bin")
    write_scene(path, scenegen.quad_scene(0.2))
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1:verify_asan_link_order=0:exitcode=99"
    r = subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 99 and "AddressSanitizer" in r.stderr, (r.returncode, r.stderr[-2000:])


ASAN_ENV = {
    "ASAN_OPTIONS": "halt_on_error=1:detect_leaks=1:verify_asan_link_order=0:exitcode=99",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=98",
}
# allocations the HIP and HSA runtimes keep until the process ends
LEAK_SUPPRESSIONS = ["leak:libamdhip64.so", "leak:libhsa-runtime64.so", "leak:libhsakmt", "leak:libdrm",
                     "leak:librocprofiler", "leak:libnuma"]


def run_host_check(exe, tmp_path, *args, timeout=120):
    sup = tmp_path / "lsan.supp"
    sup.write_text("\n".join(LEAK_SUPPRESSIONS) + "\n")
    env = dict(os.environ)
    env.update(ASAN_ENV)
    env["LSAN_OPTIONS"] = f"suppressions={sup}:print_suppressions=0"
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=timeout)
    report = r.stdout + r.stderr
    assert "runtime error" not in report and "Sanitizer" not in report, report[-6000:]
    assert r.returncode == 0, report[-6000:]
    return r.stdout


def test_host_runtime_validation_under_asan_ubsan(tmp_path):
    """Every entry point's argument checks, in host code built with the
    sanitizers (built here if build_sanitized has not run)."""
    exe = hipbuild.ASAN_CHECK
    if not os.path.exists(exe):
        if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
            pytest.skip("hipcc not found")
        _, exe = hipbuild.build_sanitized(out_dir=str(tmp_path / "asan"))
    out = run_host_check(exe, tmp_path)
    assert "validation ok" in out


@pytest.mark.gpu
def test_host_runtime_device_paths_under_asan_ubsan(tmp_path):
    """The sanitized host code driving every entry point on the GPU: scene
    builds with forced allocation failures, renders in both engines and all
    three mappings, single passes, the instrumented render, a batch, the
    allocation-free render, both autotuners, a graph, the server, ray
    generation and tracing, the sort and the screen-space passes."""
    exe = hipbuild.ASAN_CHECK
    assert os.path.exists(exe), "the sanitized driver is not built (paper_2312_12392_amd.build.build_sanitized)"
    print("[case] sanitized host driver --device", flush=True)
    out = run_host_check(exe, tmp_path, "--device", timeout=300)
    assert "validation and device paths ok" in out
