"""Stability of the collision variants (Section 3 prefers MRT for stability): a reduced map
over mobility and regularisation strength, alpha = 0.3, computed with the ensemble.

Measured (64^2 eq 40 droplet, R = 16, D = 5, 30000 steps, FP32): MRT with unit free rates
is stable at more points than SRT, and wherever SRT is except at M = 0.1 (s_j = 1.25),
where SRT also survives eps_reg = 2; TRT with magic 1/4 is stable wherever MRT is."""
import pytest

pytestmark = pytest.mark.gpu


def test_collision_stability_map():
    from paper_2501_03759_amd import stability
    mobilities, eps_regs = (0.01, 0.1, 1.0, 2.0), (0.03, 0.3, 1.0, 2.0)
    res = stability.stability_map(models=("mrt", "srt", "trt"), mobilities=mobilities, eps_regs=eps_regs,
                                  steps=30000)
    st = {(r["model"], r["mobility"], r["eps_reg"]): r["stable"] for r in res}
    print("case map\n" + stability.table(res), flush=True)
    count = {m: sum(v for (k, _, _), v in st.items() if k == m) for m in ("mrt", "srt", "trt")}
    for model in ("mrt", "srt", "trt"):
        assert st[(model, 0.1, 0.03)]                       # the eq 39 point
    assert count["mrt"] > count["srt"], count
    for m in (0.01, 1.0, 2.0):                              # away from s_j = 1.25
        srt = {e for e in eps_regs if st[("srt", m, e)]}
        mrt = {e for e in eps_regs if st[("mrt", m, e)]}
        assert srt < mrt, (m, srt, mrt)                     # strictly larger for MRT
    assert all(st[("trt", m, e)] for m in mobilities for e in eps_regs if st[("mrt", m, e)])
    assert not all(st.values())                             # the map has an edge
