"""lbm_mass_all_noalloc, the entry point that allocates nothing, against
lbm_mass (one simulation per call, accumulators in the context's workspace):
two calls in a row, the second on a context with fewer simulations, so that
stale accumulators of the first would show; and a context beyond its fixed
scratch is rejected with LBM_ERANGE."""
import numpy as np
import pytest

from paper_2505_10171_amd import workloads as W

pytestmark = pytest.mark.gpu


def _members(n, L0=20):
    out = []
    for i in range(n):
        L = L0 + 2 * i
        cfg = W.config(L, L, L, theta_wall_deg=70.0 + 5 * i, body_force=(2e-6, 0.0, 0.0))
        phi0 = W.drop_phi0(L, L, L, (L / 3.0, L / 2.0, 0.5), L / 4.0)
        parts = [W.particle((L / 2.0 + 3.0, L / 2.0, 4.0), 2.5, theta_deg=60.0,
                            sigma=cfg["sigma"])] if i % 2 == 0 else []
        out.append(dict(cfg=cfg, phi0=phi0, particles=parts))
    return out


def _check(ctx, n):
    m_static = ctx.mass_all_noalloc()
    assert m_static.shape == (n, 2)
    for i in range(n):
        m = ctx.mass(i)
        err = np.abs(m_static[i] - m) / np.abs(m)
        print(f"sim {i}: noalloc {m_static[i]} lbm_mass {m} rel {err}", flush=True)
        assert np.all(err <= 1e-12), (i, m_static[i], m)


def test_noalloc_mass_matches_lbm_mass():
    from paper_2505_10171_amd.lbm import Context
    big = Context(_members(5))
    big.step(30)
    _check(big, 5)
    big.close()
    small = Context(_members(2, L0=24))
    small.step(17)
    _check(small, 2)
    small.close()


def test_noalloc_rejects_too_many_simulations():
    from paper_2505_10171_amd.lbm import Context, LbmError, LBM_ERANGE
    ms = [dict(cfg=W.config(4, 4, 4), phi0=None, particles=[]) for _ in range(1025)]
    ctx = Context(ms)
    with pytest.raises(LbmError) as e:
        ctx.mass_all_noalloc()
    assert e.value.code == LBM_ERANGE
    ctx.close()
