"""The batched sweep's own workload at full size -- the 64-lattice droplet draw (seed 0: sides
128-1008, 23.9 M nodes, R = n/4, tau in [0.6, 1.5], T/Tc in [0.5, 0.9], BGK or MRT, Guo + Li
forcing, K = 1/49) in the launch the batched sweep and the bench time (two steps per launch,
256-thread workgroups, automatic segment heights) -- against the FP64 oracle on sampled
windows of three members after 100 steps.  Bar: 1e-5 relative in rho (pointwise) and in v
(max |dv| over the windows / max |v_ref|)."""
import numpy as np
import pytest

import oracle as O
from lbm_cases import oracle_params, say
from oracle import thermo as TH
from paper_1412_5170_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
K = 100                 # steps: 50 two-step launches
WIN = 16
MARGIN = 2 * K + 1      # one step moves information at most two nodes


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_5170_amd import lbm
    return lbm


def _rho0(m):
    g, l, _ = TH.maxwell(m["T_over_Tc"])
    return inputs.droplet(m["nx"], m["ny"], m["R"], 5.0, l, g)


def _params(m, n):
    from paper_1412_5170_amd import sweep
    return oracle_params(dict(m, nx=n, ny=n, s5=sweep.PHYSICS["s"]))


def _window(m, rho0, x0, y0):
    """Oracle fields of the WIN x WIN window at (x0, y0) after K steps: the patch with a margin
    of MARGIN around it, mirrored into a 2 x 2 periodic tile so that its seams are continuous;
    nothing from the seams reaches the window in K steps."""
    n = WIN + 2 * MARGIN
    nx, ny = m["nx"], m["ny"]
    xs = np.arange(x0 - MARGIN, x0 - MARGIN + n) % nx
    ys = np.arange(y0 - MARGIN, y0 - MARGIN + n) % ny
    P = rho0[np.ix_(ys, xs)]
    Q = np.block([[P, P[:, ::-1]], [P[::-1, :], P[::-1, ::-1]]])
    p = _params(m, 2 * n)
    fl = O.fields(p, O.step(p, O.init_feq(Q), K))
    inner = np.s_[MARGIN:MARGIN + WIN, MARGIN:MARGIN + WIN]
    return (np.ix_(ys[MARGIN:MARGIN + WIN], xs[MARGIN:MARGIN + WIN]),
            fl["rho"][inner], fl["vx"][inner], fl["vy"][inner])


def test_full_draw_sampled_windows(L):
    from paper_1412_5170_amd import sweep
    members = sweep.members_from_draw(inputs.batch_draw(0))
    assert len(members) == 64 and sum(m["nx"] * m["ny"] for m in members) == 23_917_568
    say(f"[batch full size] 64 lattices, two steps per launch, {K} steps")
    b = L.Batch(members)   # the batched sweep's launch: tx 256, two steps per launch
    rho0 = [_rho0(m) for m in members]
    for i in range(len(members)):
        b.init(i, rho0[i])
    b.step(K)
    order = sorted(range(len(members)), key=lambda i: members[i]["nx"])
    picks = [order[-1], order[len(order) // 2], order[0]]   # largest, median, smallest side
    e_rho, dv, vref = 0.0, 0.0, 0.0
    for i in picks:
        m = members[i]
        rho_g, u_g = b.read(i)
        n, c, R = m["nx"], m["nx"] // 2, int(m["R"])
        say(f"    member {i}: {n}x{n} T/Tc {m['T_over_Tc']:.3f} tau {m['tau']:.3f} "
            f"{m['collision']}")
        if n <= WIN + 2 * MARGIN:   # small: the whole lattice
            p = _params(m, n)
            fl = O.fields(p, O.step(p, O.init_feq(rho0[i]), K))
            wins = [(np.s_[:, :], fl["rho"], fl["vx"], fl["vy"])]
        else:
            # the interface on +x, on the diagonal, at +y on a strip and segment corner of
            # the two-step tiles (58 output columns, 16-row segments), and the periodic wrap
            xc = (c // 58) * 58
            wins = [_window(m, rho0[i], x0, y0) for x0, y0 in
                    ((c + R - WIN // 2, c - WIN // 2),
                     (c + int(R / 2 ** 0.5) - WIN // 2, c + int(R / 2 ** 0.5) - WIN // 2),
                     (xc - WIN // 2, ((c + R) // 16) * 16 - WIN // 2),
                     (n - WIN // 2, n - WIN // 2))]
        for sel, r_o, vx_o, vy_o in wins:
            e = float(np.max(np.abs(rho_g[sel] - r_o) / r_o))
            d = max(np.abs(u_g[sel][..., 0] - vx_o).max(), np.abs(u_g[sel][..., 1] - vy_o).max())
            e_rho, dv = max(e_rho, e), max(dv, d)
            vref = max(vref, np.abs(vx_o).max(), np.abs(vy_o).max())
            say(f"      rho {e:.3e}  |dv| {d:.3e}  max |v| "
                f"{max(np.abs(vx_o).max(), np.abs(vy_o).max()):.3e}")
    say(f"    all windows: rho {e_rho:.3e}  v {dv / vref:.3e}")
    assert e_rho < TOL and dv / vref < TOL
