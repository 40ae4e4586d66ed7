"""The product planner's device code run on the CPU (no GPU needed).

The planner section of paper_2205_08941_amd/csrc/product.hip is compiled with
g++ as host code (one-thread launches emulated by loops, tests/host/planner_main.cpp)
and run on oracle patterns of a displaced 216-atom cell: for every tile height,
both column orders, one- and two-wave tiles, transposed plans and several
numbers of planner threads per tile (up to more than the atoms), each scheduled
triple must be a real one with its A, B and C slots, every C slot must sit at
exactly one tile position, each tile's entries must run in ascending k with
padding only at the end, and the number of triples must equal the oracle's
count_triples.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM = """#include <cstdint>
#include <cstdlib>
#include <vector>
#include <algorithm>
using std::min;
using std::max;
#define __global__ static
#define __device__
#define __restrict__
struct Dim3 { int x; };
static Dim3 blockIdx, blockDim, threadIdx;
constexpr int kMaxRows = 16;
static unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) { auto o = *p; *p += v; return o; }
static int __popc(unsigned v) { return __builtin_popcount(v); }
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    src = open(os.path.join(ROOT, "paper_2205_08941_amd", "csrc", "product.hip")).read()
    a = src.index("// ---------------------------------------------------------------- planner")
    b = src.index("__global__ __launch_bounds__(1024) void k_scan64")
    main = open(os.path.join(ROOT, "tests", "host", "planner_main.cpp")).read()
    d = tmp_path_factory.mktemp("planner")
    cpp = d / "planner_host.cpp"
    cpp.write_text(SHIM + src[a:b] + main)
    exe = d / "planner_host"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(cpp)], check=True)
    return exe, d


@pytest.fixture(scope="module")
def patterns(planner):
    _, d = planner
    s = synth.make_system("d3", (3, 3, 3), 4, synth.SMALL_CUTOFFS, 6, displacement_sigma=0.1)
    out = {}
    for r in (4.0, 5.0, 7.0):
        P = O.create_pattern(s.positions, s.box, r)
        fn = d / f"p{r}.bin"
        with open(fn, "wb") as f:
            np.array([P.natoms, P.nnz], np.int32).tofile(f)
            P.rowptr.astype(np.int32).tofile(f)
            P.cols.astype(np.int32).tofile(f)
        out[r] = (P, fn)
    return out


CASES = [(7.0, 4.0, 5.0), (4.0, 7.0, 5.0), (5.0, 5.0, 7.0), (7.0, 5.0, 4.0)]


@pytest.mark.parametrize("G,JT,W,order,tr,nch", [(8, 7, 1, 1, 0, 4), (8, 7, 1, 0, 0, 4), (4, 7, 1, 1, 0, 1),
                                                  (2, 7, 1, 1, 0, 3), (16, 7, 1, 1, 0, 4), (8, 16, 1, 1, 0, 4),
                                                  (8, 7, 2, 1, 0, 4), (4, 16, 2, 1, 0, 2), (8, 7, 1, 1, 1, 4),
                                                  (4, 7, 1, 0, 1, 5), (8, 16, 1, 1, 1, 4), (8, 7, 1, 1, 0, 300)])
def test_planner_schedules_each_triple_once(planner, patterns, G, JT, W, order, tr, nch):
    exe, _ = planner
    for ra, rb, rc in CASES:
        (PA, fa), (PB, fb), (PC, fc) = patterns[ra], patterns[rb], patterns[rc]
        r = subprocess.run([str(exe), str(fa), str(fb), str(fc), str(G), str(JT), str(W), str(order), str(tr),
                            str(nch)], capture_output=True, text=True, timeout=120)
        seen, bad = (int(v) for v in r.stdout.split())
        assert r.returncode == 0 and bad == 0, (ra, rb, rc, r.stdout)
        assert seen == int(O.count_triples(PA, PB, PC).sum()), (ra, rb, rc)
