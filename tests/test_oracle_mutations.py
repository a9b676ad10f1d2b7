"""The oracle's pins catch plausible mistakes: each case compiles a copy of
oracle.c with one planted mistake (a wrong constant, a swapped operand, a
dropped or misplaced draw, a wrong particle type) and requires the named pins
(oracle_pins.py) to fail on it.  The oracle as built passes the same pins
(test_oracle_compton.py)."""
import pytest

import oracle_pins as pins

FP64 = 0

# (what, text in oracle.c (must occur exactly once), replacement, pins that must fail)
MUTATIONS = [
    ("Compton photon cut taken as the e+- cut",
     "if (Ep < kCUTG) {", "if (Ep < kCUTE) {",
     [lambda L: pins.compton_kill_and_spectrum(L, 0.5, FP64), lambda L: pins.compton_hand_trace(L, FP64)]),
    ("Compton: the photon keeps the electron's share",
     "    nl = -or_log(or_u01(b[0]));\n    Enew = Ep;", "    nl = -or_log(or_u01(b[0]));\n    Enew = T;",
     [lambda L: pins.compton_hand_trace(L, FP64), lambda L: pins.compton_kill_and_spectrum(L, 0.5, FP64)]),
    ("Compton: the electron gets the photon's share",
     "create(S, &X, OR_ELECTRON, T, t->pos, t->dir, v1, out);\n    nl = -or_log(",
     "create(S, &X, OR_ELECTRON, Ep, t->pos, t->dir, v1, out);\n    nl = -or_log(",
     [lambda L: pins.compton_hand_trace(L, FP64), lambda L: pins.compton_kill_and_spectrum(L, 0.5, FP64)]),
    ("Compton resample drawn from the wrong word (a0)",
     "    nl = -or_log(or_u01(b[0]));\n    Enew = Ep;", "    nl = -or_log(or_u01(a[0]));\n    Enew = Ep;",
     [lambda L: pins.compton_hand_trace(L, FP64)]),
    ("Compton resample dropped",
     "    nl = -or_log(or_u01(b[0]));\n    Enew = Ep;", "    nl = 0.0;\n    Enew = Ep;",
     [lambda L: pins.resample_after_compton(L, FP64), lambda L: pins.compton_hand_trace(L, FP64)]),
    ("bremsstrahlung resample dropped",
     "    nl = -or_log(or_u01(b[0]));\n    E = E2;", "    nl = 0.0;\n    E = E2;",
     [lambda L: pins.resample_after_brem(L, FP64)]),
    ("Compton ejects a positron",
     "create(S, &X, OR_ELECTRON, T, t->pos, t->dir, v1, out);\n    nl = -or_log(",
     "create(S, &X, OR_POSITRON, T, t->pos, t->dir, v1, out);\n    nl = -or_log(",
     [lambda L: pins.ledger_mixed_shower(L, FP64)]),
    ("annihilation makes one photon",
     "  create(S, X, OR_GAMMA, Eg, pos, md, v, out);\n", "",
     [lambda L: pins.ledger_mixed_shower(L, FP64)]),
    ("pair production makes two electrons",
     "create(S, &X, OR_POSITRON, Tp, t->pos, t->dir, v1, out);\n    return 0;\n  }\n  double Enew",
     "create(S, &X, OR_ELECTRON, Tp, t->pos, t->dir, v1, out);\n    return 0;\n  }\n  double Enew",
     [lambda L: pins.ledger_mixed_shower(L, FP64)]),
    ("divergence groups of 128 sources",
     "if ((i & 63) == 63 || i + 1 == S->n[D]) {", "if ((i & 127) == 127 || i + 1 == S->n[D]) {",
     [lambda L: pins.divergence_groups(L)]),
    ("divergence count includes the most common outcome",
     "S->led.off_mode += all - most;", "S->led.off_mode += all;",
     [lambda L: pins.divergence_groups(L)]),
]


@pytest.mark.parametrize("what,old,new,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(oracle_mod, tmp_path, what, old, new, checks):
    src = open(oracle_mod.SRC).read()
    assert src.count(old) == 1, what
    mutated = tmp_path / "oracle.c"
    mutated.write_text(src.replace(old, new))
    L = oracle_mod.load(oracle_mod.build(force=True, src=str(mutated), out=str(tmp_path / "liboracle_mut.so")))
    for check in checks:
        with pytest.raises(AssertionError):
            check(L)
