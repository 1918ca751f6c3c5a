"""The C-ABI library loads and exports every symbol include/lidarseg.h declares
(no device calls: these run on the CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lidar_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2005_02704_amd as lp
    from paper_2005_02704_amd.lidarserve import SERVE_EXPORTS
    L = lp.load_library()
    assert set(_declared("lidarseg.h")) == set(lp.EXPORTS)
    assert set(_declared("lidarserve.h")) == set(SERVE_EXPORTS)
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["lidarseg.h", "lidarserve.h"]
    for name in list(lp.EXPORTS) + list(SERVE_EXPORTS):
        assert hasattr(L, name), name


def test_query_sizes_and_validation_on_host():
    import paper_2005_02704_amd as lp
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 1800, 1)
    assert lp.lidar_query_sizes(geo) == (16 * 1800, 2 * 15 * 1800)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 1800, 7)   # 7 does not divide 1800
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(-15, 15, 16)), 1800, 1)   # ascending
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 200)), 1800, 1)  # too many rings
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)
    geo = lp.SensorGeometry(np.radians(np.linspace(15, -15, 16)), 2, 1, wrap=1)
    with pytest.raises(lp.LidarError):
        lp.lidar_query_sizes(geo)


def test_binding_structs_match_the_header(tmp_path):
    """Every field offset and struct size of the ctypes binding equals the C
    compiler's for include/lidarseg.h."""
    import subprocess
    from paper_2005_02704_amd import lidarseg as b
    from paper_2005_02704_amd import lidarserve as sv
    structs = [b.lidar_sensor_t, b.lidar_frame_t, b.lidar_params_t, b.lidar_result_t, sv.lidar_server_opts_t,
               sv.lidar_served_t, sv.lidar_server_result_t, sv.lidar_server_stats_t]
    lines = []
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in st._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"lidarseg.h\"\n#include \"lidarserve.h\"\n"
                   "int main(void) {\n"
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[f"{name} size"]) == ctypes.sizeof(st), name
        for fname, _ in st._fields_:
            assert int(got[f"{name} {fname}"]) == getattr(st, fname).offset, (name, fname)


def test_binding_refuses_to_run_without_the_library(tmp_path):
    """The product path has no fallback: without the built library, creating a
    context raises instead of computing anything elsewhere."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2005_02704_amd.lidarseg as L\n"
            "try:\n"
            "    L.load_library(%r)\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n"
            "    raise SystemExit(0)\n"
            "raise SystemExit(1)\n") % (ROOT, str(tmp_path / "missing.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "refused" in r.stdout


def test_binding_constants_match_the_header():
    """Every #define of include/lidarseg.h that the binding restates has the
    header's value (evaluated by the C compiler)."""
    import subprocess
    import tempfile
    import paper_2005_02704_amd as lp
    from paper_2005_02704_amd import lidarserve as sv
    names = ["LIDAR_OK", "LIDAR_EINVAL", "LIDAR_ENOMEM", "LIDAR_EDEVICE", "LIDAR_MAX_RINGS", "LIDAR_LAUNCH_PLAIN",
             "LIDAR_LAUNCH_BATCHED", "LIDAR_LAUNCH_GRAPH", "LIDAR_PRED_COMPONENTS", "LIDAR_PRED_COSINE",
             "LIDAR_MAX_SCORE_RADIUS", "LIDAR_N_STAGES", "LIDAR_NOALLOC_SCRATCH_BYTES", "LIDAR_NOALLOC_MAX_FRAMES"]
    served = ["LIDAR_SERVED_OK", "LIDAR_SERVED_TIMED_OUT", "LIDAR_SERVED_FAILED"]
    body = "\n".join(f'printf("{n} %lld\\n", (long long)({n}));' for n in names + served)
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "consts.c")
        exe = os.path.join(d, "consts")
        open(src, "w").write("#include <stdio.h>\n#include \"lidarserve.h\"\nint main(void) {\n" + body +
                             "\nreturn 0;\n}\n")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for n in names:
        assert int(got[n]) == getattr(lp, n), n
    for n in served:
        assert int(got[n]) == getattr(sv, n), n
