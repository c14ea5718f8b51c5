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
    ("sync.c", "(dv == dw && v < w)", "(dv == dw && v > w)"),                            # tie-break
    ("sync.c", "dv < dw - 1", "dv < dw + 1"),                                            # ownership rule
    ("sync.c", "if (dcur == dw + 1) {", "if (d0 == dw + 1) {"),                          # d' vs d
    ("sync.c", "if (M->cf[g->rev[a]] > 0) {          /* w can send to v */",
     "if (M->cf[a] > 0) {"),                                                             # BFS direction
    ("sync.c", "M->cf[M->blist[i]] += M->back[M->blist[i]];", "(void)0;"),               # lost reverse residual
    ("sync.c", "M->change[v] += left - M->exc[v];", "M->change[v] = left - M->exc[v];"), # '=' for the excess sum
    ("sync.c", "dw >= dcur && dw + 1 < lowest", "dw > dcur && dw + 1 < lowest"),         # raise candidate bound
    ("sync.c", "if (dcur == n || simple) break;", "if (dcur == n) break;"),              # simple: full discharge
    ("sync.c", "depth = bfs_labels(M, sink, other);", "bfs_labels(M, sink, other);"),    # level charge dropped
    ("sync.c", "if (lost[i] > 0 && lost[i] < gap && M->count[lost[i]] == 0) gap = lost[i];",
     "if (lost[i] > 0 && M->count[lost[i]] == 0) gap = lost[i];"),                      # gap: not the smallest
    ("sync.c", "if (M->lab[v] > gap && M->lab[v] < n) {",
     "if (M->lab[v] > gap + 1 && M->lab[v] < n) {"),                                    # gap: lift off by one
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
