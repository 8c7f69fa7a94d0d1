"""The ABI tests again, against a build whose host code runs under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed: every call
they make is rejected before any device work).  The sanitizer build is made
by ``paper_2212_07679_amd/build_asan.py`` (also run by
``__graft_entry__.build()``) and rebuilt here when a source is newer."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(ROOT, "paper_2212_07679_amd", "csrc", f)
            for f in os.listdir(os.path.join(ROOT, "paper_2212_07679_amd", "csrc"))]
    srcs += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return any(os.path.getmtime(s) > t for s in srcs)


def test_abi_under_address_and_undefined_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2212_07679_amd import build_asan

    if _stale(build_asan.LIB):
        build_asan.build()
    log = tmp_path / "san"
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": build_asan.asan_runtime(),
        "ASAN_OPTIONS": f"detect_leaks=0:halt_on_error=1:log_path={log}",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={log}",
        "SNN_LIBRARY": build_asan.LIB,
    })
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = "".join(p.read_text() for p in tmp_path.iterdir() if p.name.startswith("san"))
    assert r.returncode == 0 and not reports, f"{r.stdout[-3000:]}\n{r.stderr[-3000:]}\n{reports[:4000]}"
    assert " passed" in r.stdout
