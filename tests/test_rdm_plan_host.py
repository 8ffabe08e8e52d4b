"""Host check of the reduced-density-matrix pass plans (rdm.hip), compiled with hipcc and run on
the CPU (no GPU).

The check builds every pass plan for L = 2..30 and replays the quad enumeration that each wave
program of the pair kernel performs: cube items (triangles and stars of pairs over three bits,
eight amplitudes per base), single pairs (one or two quads per round), rows split between copies
of a wave or between a wave and a helper, and the slot and swap bookkeeping. It checks that:

- every quad of every pair (its four amplitudes at one base with the pair's bits clear) is
  accumulated exactly once, into a slot that holds that pair;
- the slot's swap flag says whether the quad lists the pair's higher bit first;
- every pair of bits is in exactly one pass.

The single-site plans must evaluate every bit exactly once, with the tile bits and the other bits
a partition of 0..L-1."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_10052_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

DRIVER = r'''
#include "rdm.hip"
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
namespace ed {
ed_status fail(ed_status s, const std::string&) { return s; }
bool sym_eig_jacobi(int, double*, double*, double*) { return false; }
}
using namespace ed;

static void die(const char* what, int L) { std::printf("FAIL L=%d: %s\n", L, what); std::exit(1); }

static void check_pairs(int L) {
    const std::vector<RdmPass> ps = rdm_plan(L);
    std::map<std::pair<int, int>, int> seen;
    for (const RdmPass& pa : ps) {
        const bool full = pa.T == kTileBits;
        const int tsize = 1 << pa.T;
        std::vector<std::vector<int>> cover(pa.npairs, std::vector<int>(tsize, 0));
        for (int w = 0; w < kWaves; ++w) {
            const int lay = pa.layout[w], piece = pa.piece[w], ns = pa.nsplit[w];
            auto add = [&](int S, int x0, int first, int second) {
                const int pr = pa.wpair[w][S];
                if (pr < 0) die("quad into an empty slot", L);
                const int lo = std::min(first, second), hi = std::max(first, second);
                if (pa.lp[pr] != lo || pa.lq[pr] != hi) die("slot holds another pair", L);
                if (pa.wswap[w][S] != (first > second)) die("swap flag", L);
                if (((x0 >> lo) & 1) || ((x0 >> hi) & 1)) die("base with the pair's bits set", L);
                cover[pr][x0]++;
            };
            auto one = [&](int S, int lp, int lq) {
                const int rows = full ? (1 << (kTileBits - 2)) / 64 : ((tsize >> 2) + 63) / 64;
                for (int lane = 0; lane < 64; ++lane)
                    for (int r = piece; r < rows; r += ns) {
                        if (!full && lane + 64 * r >= (tsize >> 2)) continue;
                        add(S, insert_two(lane, lp, lq) | insert_two(64 * r, lp, lq), lp, lq);
                    }
            };
            auto cube = [&](bool tri, int S0, const int* bits) {
                const int a = bits[0], b = bits[1], c = bits[2];
                if (a == b || b == c || a == c) die("cube bits repeat", L);
                const int lo = std::min(a, std::min(b, c)), hi = std::max(a, std::max(b, c)), mid = a + b + c - lo - hi;
                for (int lane = 0; lane < 64; ++lane)
                    for (int r = piece; r < (1 << (kTileBits - 3)) / 64; r += ns) {
                        const int x = insert_three(lane, lo, mid, hi) | insert_three(64 * r, lo, mid, hi);
                        add(S0, x, a, b);
                        add(S0, x + (1 << c), a, b);
                        add(S0 + 1, x, a, c);
                        add(S0 + 1, x + (1 << b), a, c);
                        if (tri) {
                            add(S0 + 2, x, b, c);
                            add(S0 + 2, x + (1 << a), b, c);
                        }
                    }
            };
            const auto& ib = pa.ib[w];
            if (lay == kLayNone) {
                for (int k = 0; k < 4; ++k)
                    if (pa.wpair[w][k] >= 0) die("idle wave holds a pair", L);
                continue;
            }
            if (!full && lay != kLayOnes) die("cube item in a partial tile", L);
            if (lay == kLayTriOne) {
                cube(true, 0, ib[0]);
                if (pa.wpair[w][3] >= 0) one(3, ib[1][0], ib[1][1]);
            } else if (lay == kLayCubeCube) {
                cube(false, 0, ib[0]);
                if (pa.wpair[w][2] >= 0) cube(false, 2, ib[1]);
            } else if (lay == kLayCubeOneOne) {
                cube(false, 0, ib[0]);
                if (pa.wpair[w][2] >= 0) one(2, ib[1][0], ib[1][1]);
                if (pa.wpair[w][3] >= 0) one(3, ib[2][0], ib[2][1]);
            } else if (lay == kLayOnes) {
                for (int k = 0; k < 4; ++k)
                    if (pa.wpair[w][k] >= 0) one(k, ib[k][0], ib[k][1]);
            } else {
                die("unknown layout", L);
            }
        }
        for (int i = 0; i < pa.npairs; ++i) {
            for (int x = 0; x < tsize; ++x) {
                const bool base = !((x >> pa.lp[i]) & 1) && !((x >> pa.lq[i]) & 1);
                if (cover[i][x] != (base ? 1 : 0)) die("a quad is missed or counted twice", L);
            }
            const auto key = std::make_pair(pa.pos[pa.lp[i]], pa.pos[pa.lq[i]]);
            if (seen.count(key)) die("pair in two passes", L);
            seen[key] = 1;
        }
    }
    if (int(seen.size()) != L * (L - 1) / 2) die("pairs missing", L);
}

static void check_sites(int L) {
    const std::vector<Rdm1Pass> ps = rdm1_plan(L);
    std::vector<int> seen(L, 0);
    for (const Rdm1Pass& pa : ps) {
        if (pa.nbits > kTileBits || pa.ncomp + pa.T != L) die("single-site pass shape", L);
        std::vector<int> all;
        for (int i = 0; i < pa.T; ++i) all.push_back(pa.pos[i]);
        for (int i = 0; i < pa.ncomp; ++i) all.push_back(pa.comp[i]);
        std::sort(all.begin(), all.end());
        for (int i = 0; i < L; ++i)
            if (all[i] != i) die("tile and other bits are not a partition", L);
        for (int i = 0; i < pa.nbits; ++i) {
            if (pa.pos[pa.lb[i]] != pa.gb[i]) die("tile bit and global bit disagree", L);
            seen[pa.gb[i]]++;
        }
    }
    for (int b = 0; b < L; ++b)
        if (seen[b] != 1) die("a site is not evaluated exactly once", L);
}

int main() {
    for (int L = 2; L <= 30; ++L) {
        check_pairs(L);
        check_sites(L);
    }
    std::printf("ok\n");
    return 0;
}
'''


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rdmplan")
    src = d / "rdm_plan_check.hip"
    src.write_text(DRIVER)
    exe = d / "rdm_plan_check"
    subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    f"-I{CSRC}", f"-I{INCLUDE}", str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    return exe


def test_rdm_plans_cover_every_quad_once(checker):
    r = subprocess.run([str(checker)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
