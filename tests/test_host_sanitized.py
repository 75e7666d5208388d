"""The library's host-side logic (host_logic.cpp: mesh validation, Morton ordering, the
treecode partition and walk) built with a host compiler under AddressSanitizer and
UndefinedBehaviorSanitizer, run on the CPU through its command-line driver
(host_check_main.cpp), and checked against the oracle: the same meshes accepted and
rejected, the same Morton order, the same far and near clusters for every batch."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import operator as O
from oracle import treecode as T
from paper_1301_5914_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1301_5914_amd", "csrc")


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("hostcheck") / "host_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(CSRC, "host_logic.cpp"),
                    os.path.join(CSRC, "host_check_main.cpp"), "-o", out], check=True)
    return out


def _run(exe, args, tmp_path, payload):
    inp = tmp_path / "in.bin"
    inp.write_bytes(payload)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, args[0], str(inp), *args[1:]], capture_output=True, text=True, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout


def _mesh_payload(xyz, nrm, tri):
    return (np.array([xyz.shape[0], tri.shape[0]], dtype=np.int32).tobytes() + np.ascontiguousarray(xyz, dtype=np.float64).tobytes()
            + np.ascontiguousarray(nrm, dtype=np.float64).tobytes() + np.ascontiguousarray(tri, dtype=np.int32).tobytes())


def test_mesh_validation_agrees_with_the_oracle(host_check, tmp_path):
    xyz, nrm, tri = inputs.icosphere(2, 2.0)
    a, b = int(tri[0, 0]), int(tri[0, 1])
    fold = nrm.copy()
    fold[[a, b]] *= -1.0
    rev = tri.copy()
    rev[5] = rev[5][::-1]
    unused = np.vstack([xyz, [[9.0, 9.0, 9.0]]]), np.vstack([nrm, [[1.0, 0.0, 0.0]]])
    flat = tri.copy()
    flat[7] = [flat[7][0], flat[7][0], flat[7][2]]
    m = inputs.molecule(20, seed=11)
    cases = {"valid": (xyz, nrm, tri), "fold": (xyz, fold, tri), "reversed": (xyz, nrm, rev),
             "open": (xyz, nrm, tri[1:]), "long_normals": (xyz, 2.0 * nrm, tri), "inward": (xyz, -nrm, tri),
             "unused_vertex": (unused[0], unused[1], tri), "repeated_vertex": (xyz, nrm, flat),
             "molecule": (m.xyz, m.nrm, m.tri)}
    for name, (x, n, t) in cases.items():
        try:
            O.validate_mesh(x, n, t)
            oracle_ok = True
        except O.MeshError:
            oracle_ok = False
        out = _run(host_check, ["mesh"], tmp_path, _mesh_payload(x, n, t)).strip()
        assert (out == "ok") == oracle_ok, (name, out)
        assert oracle_ok == (name in ("valid", "molecule")), name


def test_morton_order_agrees_with_the_oracle(host_check, tmp_path):
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000, 70000):           # both radix widths (8-bit below 65536 keys)
        pts = rng.normal(size=(n, 3))
        pts[: n // 3] = pts[0]               # ties keep the input order
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        payload = (np.array([n], dtype=np.int32).tobytes() + pts.tobytes() + lo.tobytes() + hi.tobytes())
        _run(host_check, ["morton", str(tmp_path / "out.bin")], tmp_path, payload)
        got = np.fromfile(tmp_path / "out.bin", dtype=np.int32)
        np.testing.assert_array_equal(got, T.morton_order(pts, lo, hi))


@pytest.mark.parametrize("theta,leaf,batch", [(0.7, 64, 128), (0.5, 128, 256), (0.9, 256, 512), (0.0, 64, 128)])
def test_tree_partition_agrees_with_the_oracle(host_check, tmp_path, theta, leaf, batch):
    p = inputs.kirkwood_offcenter(3)
    st = O.setup(p.xyz, p.nrm, p.tri)
    part = T.partition(st, theta, leaf, batch)
    vrank = np.empty(st.nv, dtype=np.int64)
    vrank[part.vorder] = np.arange(st.nv)
    nodes = st.y[part.torder].reshape(-1, 3)
    tgt = np.ascontiguousarray(st.xyz[part.vorder].T)            # [3][nv]
    tri = vrank[st.tri[part.torder]].astype(np.int32)
    hdr = np.array([nodes.shape[0], st.nv, st.nf, 0, leaf, batch, 2], dtype=np.int32).tobytes()
    payload = hdr + np.array([theta]).tobytes() + nodes.tobytes() + tgt.tobytes() + tri.tobytes()
    _run(host_check, ["tree", str(tmp_path / "out.txt")], tmp_path, payload)
    lines = (tmp_path / "out.txt").read_text().splitlines()
    nfar, nnear = map(int, lines[0].split())
    assert nfar == sum(len(f) for f in part.far) and nnear == sum(len(n) for n in part.near)
    for bi, line in enumerate(lines[1:1 + len(part.far)]):
        far_s, near_s = line.split("|")
        assert [int(c) for c in far_s.split()[1:]] == list(part.far[bi]), bi
        assert [int(c) for c in near_s.split()[1:]] == list(part.near[bi]), bi
    if theta == 0.0:
        assert nfar == 0
