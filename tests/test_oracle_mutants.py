"""Plant one plausible mistake at a time in the oracle (compile-time
MUT_* switches in oracle/empp_oracle.c) and check that the pins catch it.
This shows that the pins constrain every step of the oracle: the
bracket rule and its near-tie flags, the root, the reconstruction, the LW
formula, B, the superposition (its compensated sum and the excluded
source), the prior history, the pusher, the dipole, the history update,
the adaptive step and the Stage-II transport."""
import pytest

import oracle
import pins

MUTANTS = [
    "MUT_TIE_NEWER",          # ties sent to the newer half
    "MUT_KSTAR_OLDER",        # bracket one slot too old
    "MUT_ROOT_PLUS",          # the discarded '+' root of Eq. (dt)
    "MUT_ACCEL_BEFORE_RING",  # non-zero acceleration out of history
    "MUT_NO_VINTERP",         # v(t_r) = v_1 (no interpolation)
    "MUT_VPRIME_NOHAT",       # v' = c eta - v instead of c eta_hat - v
    "MUT_DROP_ACCEL",         # radiation term dropped
    "MUT_B_SIGN",             # B = E x eta_hat / c
    "MUT_DIPOLE_SIGN",        # wrong sign of the 3 (M.r) r term
    "MUT_HC_TYPO",            # u- x t in the last HC step
    "MUT_NO_FINALISE",        # newest history velocity never finalised
    "MUT_ETA_ABSOLUTE",       # eta from the rounded absolute retarded position
    "MUT_TRANSPORT_DT_NO_GAMMA",  # Stage-II step from 1/|B| without gamma
    "MUT_TRANSPORT_OLD_V",    # Stage-II drift with the velocity before the kick
    "MUT_ADAPT_NO_ALLOW",     # adaptive step ignores the eta_allow cutoff
    "MUT_ADAPT_ETA_PRESENT",  # adaptive step from the present, not retarded, distance
    "MUT_NO_NEAR_TIE",        # light-cone decisions next to the cone never flagged
    "MUT_SUM_SKIP_LAST",      # the superposition stops one source short
    "MUT_SELF_INDEX_IGNORED",  # the excluded source is summed anyway
    "MUT_NEUMAIER_SIGN",      # the compensation subtracted instead of added
    "MUT_INIT_NO_GAMMA",      # prior history moves with u instead of u / gamma
    "MUT_INIT_FORWARD",       # prior history extrapolated forward in time
]


@pytest.mark.parametrize("mutant", MUTANTS)
def test_mutant_is_caught(mutant, tmp_path):
    lib = oracle.build_mutant(mutant, str(tmp_path))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            ok, _ = pin(orc)
        except Exception:  # an exception is a failed pin as well
            ok = False
        if not ok:
            failed.append(pin.__name__)
    print(mutant, "caught by", failed)
    assert failed, f"{mutant} passes every pin"
