"""Host logic: the library's check that a body mesh is closed and consistently oriented
(every undirected edge used by exactly two triangles, once in each direction), compiled
from its header with the host compiler (plain, and with AddressSanitizer and
UndefinedBehaviorSanitizer) and run on small meshes with known answers."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(HERE, "..", "paper_2505_17287_amd", "csrc", "mesh_check.hpp")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "mesh_check.hpp"
int main() {
    long long nv, nt;
    while (std::scanf("%lld %lld", &nv, &nt) == 2) {
        std::vector<int32_t> t(3 * nt);
        for (auto &x : t) if (std::scanf("%d", &x) != 1) return 2;
        const char *why = ibm::mesh_closed_oriented(t.data(), nt, nv);
        std::printf("%s\n", why ? "refused" : "ok");
    }
    return 0;
}
"""


def _cube():
    """The 12 outward-oriented triangles of the unit cube's surface (8 vertices)."""
    quads = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (2, 3, 7, 6), (1, 2, 6, 5), (0, 4, 7, 3)]
    tris = []
    for a, b, c, d in quads:
        tris += [(a, b, c), (a, c, d)]
    return np.array(tris, dtype=np.int32)


# the plain build, and one with AddressSanitizer (leak detection on) and
# UndefinedBehaviorSanitizer, every report fatal
BUILDS = {"plain": [], "asan_ubsan": ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                      "-fno-sanitize-recover=undefined"]}


@pytest.fixture(scope="module", params=sorted(BUILDS))
def checker(tmp_path_factory, request):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("meshcheck")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O1", "-std=c++17", *BUILDS[request.param], "-I", os.path.dirname(HDR), str(src),
                    "-o", str(exe)], check=True)

    def run(cases):
        text = "".join("%d %d %s\n" % (nv, len(t), " ".join(map(str, np.asarray(t).ravel()))) for nv, t in cases)
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split()
        return out

    return run


def test_mesh_check_verdicts(checker):
    cube = _cube()
    flipped = cube.copy()
    flipped[3] = flipped[3][::-1]
    missing = cube[1:]
    duplicated = np.vstack([cube, cube[:1]])
    degenerate = cube.copy()
    degenerate[0, 1] = degenerate[0, 0]
    two = np.vstack([cube, cube + 8])  # two disjoint closed cubes
    twisted = np.vstack([cube, (cube + 8)[:, ::-1]])  # the second one inward: still consistent
    cases = [(8, cube), (8, flipped), (8, missing), (8, duplicated), (8, degenerate), (16, two), (16, twisted),
             (16, np.vstack([cube, cube]))]
    assert checker(cases) == ["ok", "refused", "refused", "refused", "refused", "ok", "ok", "refused"]


def test_mesh_check_workload_meshes(checker):
    """The benchmark and test bodies pass; each with one triangle flipped is refused."""
    from paper_2505_17287_amd import inputs as I
    cases = []
    for wl in (I.multibody(64), I.wing(64, 32, 32)):
        t = np.ascontiguousarray(wl.tris, dtype=np.int32)
        bad = t.copy()
        bad[len(bad) // 2] = bad[len(bad) // 2][::-1]
        cases += [(len(wl.verts), t), (len(wl.verts), bad)]
    assert checker(cases) == ["ok", "refused", "ok", "refused"]


def test_oracle_mesh_check_verdicts():
    """The oracle's own closedness check (orc_set_mesh) gives the same verdicts on the same
    meshes: closed and consistently oriented, or refused with ORC_E_GEOMETRY (-3); indices
    out of range are ORC_E_ARG (-1)."""
    from oracle import OracleProblem
    from oracle.oracle import OracleError
    cube = _cube()
    verts = np.array([[x, y, z] for z in (0.0, 1.0) for y in (0.0, 1.0) for x in (0.0, 1.0)])
    verts = verts[[0, 1, 3, 2, 4, 5, 7, 6]] * 0.5 - 0.2  # vertex order of _cube's quads
    flipped = cube.copy()
    flipped[3] = flipped[3][::-1]
    degenerate = cube.copy()
    degenerate[0, 1] = degenerate[0, 0]
    two_v = np.vstack([verts, verts + 0.6])
    f = np.linspace(-1.0, 1.0, 9)
    cases = [(verts, cube, 0), (verts, flipped, -3), (verts, cube[1:], -3), (verts, np.vstack([cube, cube[:1]]), -3),
             (verts, degenerate, -3), (two_v, np.vstack([cube, cube + 8]), 0), (two_v, np.vstack([cube, cube]), -3),
             (verts, np.where(cube == 7, 8, cube), -1)]
    for v, t, want in cases:
        P = OracleProblem(f, f, f)
        try:
            P.set_mesh(v, np.ascontiguousarray(t, dtype=np.int32))
            got = 0
        except OracleError as e:
            got = e.code
        assert got == want, (t.shape, got, want)
