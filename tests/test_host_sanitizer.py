"""Host code of libuot under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled for the host only (--offload-host-only: no
device code is built, kernel launches keep their host stubs; the new offload
driver's host objects carry kernel entries rather than a reference to a
device image, so they link without one) with the
sanitizers placed behind -Xarch_host, linked with the C++ driver
tests/host/host_checks.cpp against the HIP runtime, and run without a GPU.  The
driver calls the sizing and validation paths of the C ABI (plan building for
every geometry, ragged batch offsets, network layouts, NULL-context calls and
uot_create with no device) and checks the documented status codes; the
sanitizers must report nothing.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_05816_amd", "csrc")
SOURCES = ["uot_kernels.hip", "uot_grid_tf.hip", "uot_dense_mf.hip", "uot_api.hip", "uot_net.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, **kw)
    return r.returncode, r.stdout.decode(errors="replace")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs the ROCm toolchain")
def test_host_paths_clean_under_asan_ubsan(tmp_path):
    objs, procs = [], []
    for src in SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "--offload-host-only",
               "--offload-new-driver", *SAN,
               "-Wno-unused-command-line-argument", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, "host-only compile of %s failed:\n%s" % (src, out.decode(errors="replace"))
    exe = str(tmp_path / "host_checks")
    rc, out = _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "host_checks.cpp"),
                    *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert rc == 0, "link failed:\n" + out
    env = dict(os.environ)
    # the HIP runtime keeps its own allocations past exit; leaks are not what this checks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""      # no device, also on a machine that has one
    rc, out = _run([exe], env=env, timeout=120)
    assert rc == 0 and "host checks passed" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    shutil.rmtree(str(tmp_path), ignore_errors=True)
