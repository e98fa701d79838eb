"""The compile-time contact-shell and ball tables of the GPU library
(paper_1304_7880_amd/csrc/shell.hpp, which the compiled kernels and the host
quad table are built from) against the oracle's own stencils: the quads,
expanded over their mirror images with their multiplicity weights, must
cover the oracle's shell exactly once; the weights must be w * e / |e|
(w = 1, 1/2, 1/4); the ball must equal the oracle's ball, in z, y, x order.
CPU only: the header is plain C++ and is compiled here with g++.
"""
import decimal
import json
import os
import shutil
import subprocess
from collections import Counter
from fractions import Fraction

import pytest

from oracle import ref

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1304_7880_amd", "csrc")
S2S = (6, 8, 12, 16, 20)

PROGRAM = r"""
#include <cstdio>
#include "shell.hpp"
using namespace wdlb;
template <int S2> void dump() {
    using SH = Shell<S2>;
    using B = Ball<S2>;
    std::printf("{\"s2\": %d, \"R\": %d, \"qs\": [", S2, SH::R);
    for (int k = 0; k < 2 * SH::R + 2; ++k) std::printf("%s%d", k ? ", " : "", SH::T.qs[k]);
    std::printf("], \"quads\": [");
    for (int k = 0; k < SH::NQ; ++k) {
        const CQuad &q = SH::T.q[k];
        std::printf("%s[%d, %d, %d, %d, %.17g, %.17g, %.17g, %.17g, %.17g, %.17g, %.17g, %.17g, %.17g]", k ? ", " : "",
                    q.a, q.b, q.c, q.h, q.px, q.py, q.pz, q.qxx, q.qyy, q.qzz, q.qxy, q.qxz, q.qyz);
    }
    std::printf("], \"rb\": %d, \"ball\": [", B::RB);
    for (int k = 0; k < B::NB; ++k) std::printf("%s[%d, %d, %d]", k ? ", " : "", B::T.x[k], B::T.y[k], B::T.z[k]);
    std::printf("]}\n");
}
int main() { dump<6>(); dump<8>(); dump<12>(); dump<16>(); dump<20>(); return 0; }
"""


@pytest.fixture(scope="module")
def tables(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tables")
    src, exe = d / "dump.cpp", d / "dump"
    src.write_text(PROGRAM)
    subprocess.run(["g++", "-std=c++17", "-O1", "-fconstexpr-ops-limit=100000000", "-I", CSRC, "-o", str(exe),
                    str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {t["s2"]: t for t in map(json.loads, out.strip().splitlines())}


@pytest.mark.parametrize("s2", S2S)
def test_shell_quads_cover_the_oracle_shell(tables, s2):
    t = tables[s2]
    sigma = s2 / 2.0
    covered = Counter()
    for a, b, c, h, *_ in t["quads"]:
        w = (1.0 if a > 0 else 0.5) * (1.0 if b > 0 else 0.5)
        for sa, sb in ((a, b), (-a, b), (a, -b), (-a, -b)):
            covered[(sa, sb, c)] += w
        assert h == (a & 1) | ((b & 1) << 1) | ((c & 1) << 2)
    shell = {tuple(map(int, e)) for e in ref.shell(sigma)}
    assert set(covered) == shell
    assert all(abs(v - 1.0) < 1e-15 for v in covered.values())
    assert t["R"] == max(abs(e[0]) for e in shell)
    # quads sorted by c, with qs the start of each c
    cs = [q[2] for q in t["quads"]]
    assert cs == sorted(cs)
    for k, c in enumerate(range(-t["R"], t["R"] + 1)):
        assert cs[t["qs"][k]:t["qs"][k + 1]] == [c] * (t["qs"][k + 1] - t["qs"][k])


@pytest.mark.parametrize("s2", S2S)
def test_shell_weights_are_unit_vectors_times_multiplicity(tables, s2):
    """Each coefficient against its exact value, w e_i / |e| (40 digits) and
    w e_i e_j / |e|^2 (a rational): the table's root is within an ulp, one
    division and one product add half an ulp each, so the bound is 8 unit
    roundoffs; a coefficient whose exact value is 0 must be 0."""
    decimal.getcontext().prec = 40
    u = 2.0 ** -53
    for a, b, c, h, *got in tables[s2]["quads"]:
        w = Fraction(1, (1 if a > 0 else 2) * (1 if b > 0 else 2))
        e = (a, b, c)
        r2 = a * a + b * b + c * c
        inv = 1 / decimal.Decimal(r2).sqrt()
        exact = [float(decimal.Decimal(w.numerator) / w.denominator * ei * inv) for ei in e]
        exact += [float(w * e[i] * e[j] / r2) for i, j in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))]
        for g, x in zip(got, exact):
            if x == 0.0:
                assert g == 0.0
            else:
                assert abs(g - x) <= 8 * u * abs(x), (e, g, x)


@pytest.mark.parametrize("s2", S2S)
def test_ball_equals_the_oracle_ball(tables, s2):
    t = tables[s2]
    b = [tuple(e) for e in t["ball"]]
    o = [tuple(map(int, e)) for e in ref.ball(s2 / 2.0)]
    assert b == o                      # same offsets, same z, y, x order
    assert t["rb"] == max(abs(e[0]) for e in o)
