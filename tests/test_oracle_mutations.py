"""The oracle's pins reject plausible mistakes in the oracle: each entry of
mutants.MUTANTS (a dropped term, a wrong sign, a neighbour taken from the
wrong cell, a wrong index or width, a misread coefficient formula) is
planted in a copy of rkl_oracle.c, built, and the pin files it names are
run against that copy ($RKL_ORACLE_LIB); they must fail.  CPU only."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from mutants import MUTANTS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rkl_oracle.c")


def _caught(item, src, workdir):
    name, old, new, pins = item
    d = os.path.join(workdir, name)
    os.makedirs(d)
    with open(os.path.join(d, "m.c"), "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                           "-o", os.path.join(d, "m.so"), os.path.join(d, "m.c"), "-lm"])
    env = dict(os.environ, RKL_ORACLE_LIB=os.path.join(d, "m.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + [os.path.join(ROOT, "tests", p) for p in pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # exit status 1: tests ran and failed (not a crash, an import error or no tests)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    src = open(SRC).read()
    for name, old, _, _ in MUTANTS:
        assert src.count(old) == 1, name
    with ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda m: _caught(m, src, str(tmp_path)), MUTANTS))
    missed = [(name, rc) for name, rc in results if rc != 1]
    assert not missed, missed
