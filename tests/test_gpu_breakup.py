"""Physics check against the paper's own results: break-up times of the
perturbed ligament at G_0 = -5.3, Oh = 0.1, delta = R0/10 with the Table 1
(SRT, velocity shift) and Table 2 (MRT, Guo-like forcing) parameters, against
the T_break / t_cap values of Fig. 2b.

Tolerances: 8 % at R0 = 14 and 5 % at R0 = 28.  The runs differ from the
paper's in details it does not state (initial interface profile, break-up
criterion, sampling every 25 steps); the differences shrink with R0 (below
1 % at R0 = 42 and 56, see the design notes).
"""
import pytest

pytestmark = pytest.mark.gpu

# Fig. 2b of the paper: T_break / t_cap
PAPER = {("mrt", 14): 5.925, ("mrt", 28): 6.925, ("srt", 14): 5.975, ("srt", 28): 7.375}


def test_breakup_times_match_fig2b():
    from paper_1905_09554_amd import breakup
    got = {}
    for (op, R0), ref in PAPER.items():
        t, steps, _ = breakup.break_time(R0, op)
        got[(op, R0)] = t
        print("%s R0=%d: T_break/t_cap = %.3f (paper %.3f), %d steps" % (op, R0, t, ref, steps),
              flush=True)
        tol = 0.08 if R0 == 14 else 0.05
        assert abs(t / ref - 1) < tol, (op, R0, t, ref)
    # Trends of Fig. 2b: later break-up at larger R0, SRT later than MRT.
    for op in ("mrt", "srt"):
        assert got[(op, 28)] > got[(op, 14)]
    for R0 in (14, 28):
        assert got[("srt", R0)] > got[("mrt", R0)]
