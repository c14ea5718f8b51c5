"""Each plausible mistake planted in a copy of the oracle must make some pin
fail (the pins are chosen so that a dropped term, a wrong sign or index, or
a transposed operand shows).  The copies are compiled and run on the CPU."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("sync.c", "(S->d[v] == S->d[w] && v < w)", "(S->d[v] == S->d[w] && v > w)"),       # tie-break
    ("sync.c", "(S->d[v] < S->d[w] - 1)", "(S->d[v] < S->d[w] + 1)"),                   # win rule
    ("sync.c", "int admissible = (S->dprime[v] == S->d[w] + 1);",
     "int admissible = (S->d[v] == S->d[w] + 1);"),                                      # d' vs d
    ("sync.c", "if (S->res[g->rev[a]] <= 0) continue;        /* c_f(w,v) > 0 */",
     "if (S->res[a] <= 0) continue;"),                                                   # BFS direction
    ("sync.c", "S->res[b] += S->pending[b];", "(void)0;"),                               # lost reverse residual
    ("sync.c", "S->addedExcess[v] += e - S->e[v];", "S->addedExcess[v] = e - S->e[v];"), # listing's '='
    ("sync.c", "if (S->res[a] > 0 && S->d[w] >= S->dprime[v]) {",
     "if (S->res[a] > 0 && S->d[w] > S->dprime[v]) {"),                                  # relabel candidate bound
    ("sync.c", "if (sc->simple) break;               /* simple rounds: one pass, one relabel */",
     "(void)0;"),                                                                        # simple: full discharge
    ("sync.c", "lastDepth = GlobalRelabel(S, sink, other);", "GlobalRelabel(S, sink, other);"),  # level charge dropped
    ("fifo.c", "S->res[g->rev[a]] += delta;", "(void)delta;"),                           # lost reverse residual
    ("fifo.c", "nd = S->d[g->head[a]] + 1;", "nd = S->d[g->head[a]];"),                  # relabel off by one
    ("fifo.c", "if (S->res[a] > 0 && S->d[v] == S->d[w] + 1) {",
     "if (S->res[a] > 0 && S->d[v] == S->d[w] - 1) {"),                                  # wrong sign
    ("check.c", "if (res[g->rev[a]] > 0) {          /* residual arc w -> v */",
     "if (res[a] > 0) {"),                                                               # transposed operand
]


def _build(tmp, fname, old, new):
    src = os.path.join(ROOT, "oracle")
    for f in ("oracle.h", "check.c", "fifo.c", "sync.c"):
        shutil.copy(os.path.join(src, f), tmp)
    p = os.path.join(tmp, fname)
    text = open(p).read()
    assert text.count(old) == 1, (fname, old)
    open(p, "w").write(text.replace(old, new))
    so = os.path.join(tmp, "liboracle_mut.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", so,
                    os.path.join(tmp, "check.c"), os.path.join(tmp, "fifo.c"),
                    os.path.join(tmp, "sync.c")], check=True)
    return so


def _pins(so):
    env = dict(os.environ)
    if so:
        env["ORACLE_LIB"] = so
    try:
        return subprocess.run([sys.executable, os.path.join(ROOT, "tests", "_pins_quick.py")],
                              env=env, timeout=20).returncode
    except subprocess.TimeoutExpired:
        return -1        # a mutant that never terminates fails the pins too


def test_unmodified_oracle_passes_quick_pins():
    assert _pins(None) == 0


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_planted_mistake_is_caught(idx, tmp_path):
    so = _build(str(tmp_path), *MUTANTS[idx])
    assert _pins(so) != 0, MUTANTS[idx]
