"""The Python binding's ctypes structures match the C headers byte for byte,
and the SNN_LOG environment variable reports failing calls on stderr.

A C program compiled from include/*.h prints sizeof and offsetof of every
structure the binding mirrors; the test compares them with ctypes.  No GPU
and no compute call is needed."""

import ctypes
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

from paper_2212_07679_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def mirrored_structs():
    heads = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("snn.h", "snn_testing.h"))
    out = []
    for name in dir(B):
        cls = getattr(B, name)
        if isinstance(cls, type) and issubclass(cls, ctypes.Structure) and f"}} {name};" in heads:
            out.append(cls)
    return out


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    structs = mirrored_structs()
    lines = []
    for cls in structs:
        t = cls.__name__
        lines.append(f'printf("{t} %zu\\n", sizeof({t}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    src = textwrap.dedent("""\
        #include <stddef.h>
        #include <stdio.h>
        #include "snn.h"
        #include "snn_testing.h"
        int main(void) {
        %s
          return 0;
        }
        """) % "\n".join("  " + l for l in lines)
    d = tmp_path_factory.mktemp("layout")
    c = d / "layout.c"
    c.write_text(src)
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        k, v = line.split()
        got[k] = int(v)
    return structs, got


def test_binding_mirrors_every_header_struct():
    names = {c.__name__ for c in mirrored_structs()}
    for t in ("snn_device", "snn_options", "snn_csr", "snn_stats", "snn_index_view", "snn_instance",
              "snn_batch_options", "snn_batch_info_t", "snn_screen_layout"):
        assert t in names, t


def test_struct_sizes_and_offsets_match_c(c_layout):
    structs, got = c_layout
    for cls in structs:
        t = cls.__name__
        assert ctypes.sizeof(cls) == got[t], f"sizeof({t})"
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == got[f"{t}.{f}"], f"offsetof({t}, {f})"


def test_stats_has_one_time_per_stage():
    assert len(B.snn_stats().stage_ms) == 5


def _failing_call(env_value):
    """Runs one call that fails its argument check, in a child process with
    SNN_LOG set; returns the child's stderr."""
    code = textwrap.dedent("""\
        import ctypes
        from paper_2212_07679_amd import binding as B
        out = ctypes.c_void_p()
        st = B.lib().snn_index(None, ctypes.c_void_p(0x1000), 10, 2, 0, ctypes.byref(out))
        assert st == B.SNN_EINVAL, st
        """)
    env = dict(os.environ)
    env["SNN_LOG"] = env_value
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stderr


def test_log_reports_failing_calls():
    err = _failing_call("1")
    assert "[snn] failed: SNN_EINVAL" in err, err


def test_log_is_silent_by_default():
    assert "[snn]" not in _failing_call("0")
