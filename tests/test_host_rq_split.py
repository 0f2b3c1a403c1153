"""Host checks of the index arithmetic the q-recomputing CG pass uses to split
long rows over overlapping wave windows (rq_nstrips / rq_window in
csrc/pi_common.h) and to number its boundary-layer tasks (rq_ntasks).  The
header's own functions are compiled for the host and run over every row
length up to 5000; no GPU is used.

What must hold, from the pass's dependencies (q_k at a cell needs p_{k-1}
two cells away along x, and a window zeroes what lies beyond its edges):
every lane loads four in-grid cells, each owned cell lies at least two cells
inside every window edge that is not a grid face, ownership falls on lane
boundaries, and the owned ranges tile the row exactly once."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <cstdio>
#include "pi_common.h"
int main() {
  for (int nx = 4; nx <= 5000; nx += 4) {
    const int n = pi::rq_nstrips(nx);
    std::printf("%d %d", nx, n);
    for (int xs = 0; xs < n; ++xs) {
      int start, own0, own1;
      pi::rq_window(nx, n, xs, start, own0, own1);
      std::printf(" %d %d %d", start, own0, own1);
    }
    std::printf("\n");
  }
  std::printf("tasks %lld %lld %lld %lld\n", (long long)pi::rq_ntasks(256, 256, 1), (long long)pi::rq_ntasks(500, 500, 2),
              (long long)pi::rq_ntasks(5, 6, 1), (long long)pi::rq_ntasks(23, 17, 1));
  return 0;
}
"""


@pytest.fixture(scope="module")
def split_table(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rq_split")
    src, exe = d / "split.hip", d / "split"
    src.write_text(PROGRAM)
    inc = os.path.join(ROOT, "paper_2311_16935_amd", "csrc")
    r = subprocess.run([hipcc, "-std=c++17", "-O1", "--offload-arch=gfx950", "-I", inc, "-o", str(exe), str(src)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout.splitlines()
    rows = {}
    for ln in out[:-1]:
        v = [int(x) for x in ln.split()]
        rows[v[0]] = (v[1], [tuple(v[2 + 3 * i:5 + 3 * i]) for i in range(v[1])])
    tasks = [int(x) for x in out[-1].split()[1:]]
    return rows, tasks


def test_windows_tile_each_row_with_margins(split_table):
    rows, _ = split_table
    span = 256  # 64 lanes of four cells
    for nx, (n, wins) in rows.items():
        if nx <= span:
            assert n == 1 and wins == [(0, 0, nx)]
            continue
        assert n >= 2
        assert wins[0][1] == 0 and wins[-1][2] == nx
        for (s0, a0, b0), (s1, a1, b1) in zip(wins, wins[1:]):
            assert b0 == a1, (nx, wins)  # owned ranges meet exactly
        for s, a, b in wins:
            assert a < b
            assert s % 4 == 0 and a % 4 == 0 and b % 4 == 0, (nx, s, a, b)  # lane boundaries
            assert 0 <= s and s + span <= nx, (nx, s)  # every lane's loads in the grid
            lo = s + 2 if s > 0 else 0  # cells evaluated correctly
            hi = s + span - 2 if s + span < nx else nx
            assert lo <= a and b <= hi, (nx, s, a, b)


def test_split_is_used_where_the_windows_match_the_plans_strips(split_table):
    rows, _ = split_table
    same = [nx for nx, (n, _) in rows.items() if n == (nx + 255) // 256]
    assert all(nx in same for nx in range(4, 505, 4))  # every row up to 504 cells
    assert 508 not in same and 512 not in same and 752 in same and 756 not in same
    # a window owns at most 252 cells, so k windows cover at most 504 + 248 (k - 2)
    for nx, (n, wins) in rows.items():
        if n >= 2:
            assert nx <= 504 + 248 * (n - 2)
            assert all(b - a <= 252 for _, a, b in wins)


def test_boundary_task_counts(split_table):
    _, tasks = split_table
    # 256^3: 6 boundary rows in 86 chunks of three planes + 2 face tasks for
    # each of the 250 other rows; 500^3 (two windows per row): twice
    # (6 * 167 + 2 * 494); (5, 6): no interior, every row in chunks; (23, 17)
    assert tasks == [6 * 86 + 2 * 250, 2 * (6 * 167 + 2 * 494), 5 * 2, 6 * 6 + 2 * 17]
