"""The device's exact comparison arithmetic (2304-bit two's-complement integers and the
streaming evaluator of q*Wd - pb*sum_j c_j/S_j used when two gain estimates cannot be told
apart) compiled for the host from the same source text and checked against exact Fractions:
random terms, near-ties around the decision boundary and exact ties, up to 64 slices with
2m_s < 2^31 and |c_j| up to 2^62."""
import os
import random
import shutil
import subprocess
import tempfile
from fractions import Fraction as F

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DEVICE_HPP = os.path.join(HERE, "..", "paper_2608_03695_amd", "csrc", "device.hpp")

MAIN = r"""
int main() {
  int n;
  if (scanf("%d", &n) != 1) return 1;
  for (int t = 0; t < n; t++) {
    long long q, Wd, pb;
    int m;
    if (scanf("%lld %lld %lld %d", &q, &Wd, &pb, &m) != 4) return 1;
    ExactAcc acc;
    acc.init();
    for (int j = 0; j < m; j++) {
      long long c, S;
      if (scanf("%lld %lld", &c, &S) != 2) return 1;
      acc.term(c, S);
    }
    printf("%d\n", acc.sign(q, Wd, pb));
  }
  return 0;
}
"""


def _cases(seed, n):
    rnd = random.Random(seed)
    out = []
    for _ in range(n):
        m = rnd.choice([1, 2, 3, 5, 8, 16, 32, 64])
        q = rnd.randint(1, 2**31 - 1)
        pb = rnd.randint(0, 2**62 - 1)
        terms = []
        for _ in range(m):
            S = rnd.choice([1, rnd.randint(1, 2**31 - 1), 2**31 - 1, rnd.randint(1, 100)])
            c = rnd.choice([0, rnd.randint(-2**62, 2**62), rnd.randint(-1000, 1000),
                            -(2**62), 2**62])
            terms.append((c, S))
        T = sum(F(c, S) for c, S in terms)
        r = rnd.random()
        if r < 0.1:               # exact tie: pb * c == 1 * Wd
            S = rnd.randint(1, 2**20)
            c = rnd.randint(-2**30, 2**30)
            terms, q, pb = [(c * S, S)], 1, rnd.randint(0, 2**20)
            Wd = pb * c
        elif r < 0.6:             # next to the boundary q*Wd = pb*T
            Wd = int(pb * T / q) + rnd.choice([-1, 0, 1])
            Wd = max(min(Wd, 2**62), -2**62)
        else:
            Wd = rnd.randint(-2**62, 2**62)
        T = sum(F(c, S) for c, S in terms)
        v = q * Wd - pb * T
        out.append((q, Wd, pb, terms, (v > 0) - (v < 0)))
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_exact_evaluator_matches_fractions():
    src = open(DEVICE_HPP).read()
    a = src.index("constexpr int kLimbs")
    b = src.index("// Double-precision estimate of")
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, "big.cpp")
        with open(cpp, "w") as fh:
            fh.write("#include <cstdint>\n#include <cstdio>\n#define __device__\n")
            fh.write(src[a:b])
            fh.write(MAIN)
        exe = os.path.join(d, "big")
        subprocess.run(["g++", "-O2", "-std=c++17", cpp, "-o", exe], check=True)
        cases = _cases(7, 4000)
        text = f"{len(cases)}\n" + "".join(
            f"{q} {Wd} {pb} {len(t)} " + " ".join(f"{c} {S}" for c, S in t) + "\n"
            for q, Wd, pb, t, _ in cases)
        got = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
        signs = [int(x) for x in got.stdout.split()]
        assert signs == [e for *_, e in cases]
        assert {-1, 0, 1} <= set(signs)
