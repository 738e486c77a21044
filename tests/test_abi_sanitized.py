"""The host-side ABI checks of test_abi_cpu.py, run against a build whose host code carries
AddressSanitizer and UndefinedBehaviorSanitizer (argument validation, workspace carving
with null bases, size queries, model-file parsing).  The sanitizers' runtime is preloaded
into a child Python; any report fails the child and this test."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2502_05339_amd import build
    lib = build.build_host_sanitized()
    runtime = build.asan_runtime()
    log = str(tmp_path / "san")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "DMDMI_LIBRARY": lib,
        "ASAN_OPTIONS": f"detect_leaks=0:halt_on_error=1:log_path={log}",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={log}",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"), "-q",
                        "-p", "no:cacheprovider", "-x"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    reports = "".join(open(f).read() for f in glob.glob(log + "*"))
    assert r.returncode == 0 and not reports, (r.stdout[-3000:], r.stderr[-3000:], reports[:4000])
    assert "passed" in r.stdout
