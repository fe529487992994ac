"""ht_truncate captured in a HIP graph (through torch.cuda.graph) and replayed.

The call is made once eagerly (its launch tables are uploaded and the
library's second stream and events exist), then captured on a side stream;
the plan forks to the library's second stream and joins back, so the capture
spans both streams.  Each replay, with the program's own eager work and
synchronisations between replays, must reproduce the eager result (float64
path; the split-K products add in a different order from run to run, so the
comparison is to ten times the spread of two eager runs, at least 1e-13,
rather than bit for bit) and match the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import ht_oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1708_03340_amd as H
    H.lib()
    return H


def rand_ht(rng, d, n, k):
    tr = O.Tree(d)
    U = [rng.standard_normal((n, k)) for _ in range(d)]
    B = {t: rng.standard_normal((k, k) if t == 0 else (k, k, k)) for t in range(tr.n_nodes) if not tr.is_leaf(t)}
    return O.HT(tr, U, B, 0)


def to_oracle(dev):
    U, B, s = dev.to_host()
    return O.HT(O.Tree(dev.d), U, B, s)


def test_truncate_graph_replays(H):
    import torch
    # A + C at d = 8, n = 300, k = 16 + 16, N(0,1) data, truncated to rank 12:
    # a generic spectrum, so two runs agree far below the parity gate
    say("case graph capture of ht_truncate, d=8 n=300 k=16+16 -> 12")
    rng = np.random.default_rng(5150)
    A, C = rand_ht(rng, 8, 300, 16), rand_ht(rng, 8, 300, 16)
    T, info = O.truncate(O.add(A, C), mode="fixed", ranks=[12] * 15)
    f64 = torch.float64
    devs = [H.DeviceHT.from_arrays(8, X.U, [X.B.get(t) for t in range(15)], 0, frame_dtype=f64,
                                   transfer_dtype=f64) for X in (A, C)]
    tr = H.Truncator(devs, [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=[12] * 15, precision=H.HT_PREC_FP64,
                     out_frame_dtype=f64, out_transfer_dtype=f64)
    res = tr()
    torch.cuda.synchronize()
    eager = to_oracle(res.out)
    res2 = tr()
    torch.cuda.synchronize()
    spread = O.rel_diff(to_oracle(res2.out), eager)
    say(f"  eager vs oracle {O.rel_diff(eager, T):.3e}; two eager runs differ by {spread:.3e}")
    assert O.rel_diff(eager, T) <= 1e-10
    # another truncation, run eagerly between the replays
    other = H.Truncator(devs, [1.0, -0.5], mode=H.HT_RANK_FIXED, ranks=[6] * 15, precision=H.HT_PREC_FP64,
                        out_frame_dtype=f64, out_transfer_dtype=f64)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        tr(stream=s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            tr(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for u in tr.out.leaves:          # clobber the output so a replay that writes nothing fails
            u.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = to_oracle(tr.out)
        e_eager, e_or = O.rel_diff(got, eager), O.rel_diff(got, T)
        say(f"  replay {rep}: vs eager {e_eager:.3e}, vs oracle {e_or:.3e}")
        assert e_eager <= max(1e-13, 10 * spread) and e_or <= 1e-10
        other()
        torch.cuda.synchronize()


def test_batched_truncate_graph_replays(H):
    """ht_truncate_batched over 10 uneven problems (d 4..9, n 50..300, ranks
    4..16 per summand, float64 path, fixed and tolerance rank rules),
    captured once in a HIP graph and replayed three times with eager work
    between the replays: every problem of every replay matches the eager
    batch (ten times the spread of two eager runs, at least 1e-13) and the
    oracle (1e-10)."""
    import torch
    say("case graph capture of ht_truncate_batched, 10 uneven problems")
    rng = np.random.default_rng(5151)
    f64 = torch.float64
    problems, refs = [], []
    for b in range(10):
        d, n, k = int(rng.integers(4, 10)), int(rng.integers(50, 301)), int(rng.integers(4, 17))
        A, C = rand_ht(rng, d, n, k), rand_ht(rng, d, n, k)
        nn = 2 * d - 1
        devs = [H.DeviceHT.from_arrays(d, X.U, [X.B.get(t) for t in range(nn)], 0, frame_dtype=f64,
                                       transfer_dtype=f64) for X in (A, C)]
        if b % 2 == 0:
            r = max(2, k - 2)
            problems.append(dict(Xs=devs, coef=[1.0, 0.5], mode=H.HT_RANK_FIXED, ranks=[r] * nn,
                                 precision=H.HT_PREC_FP64, out_frame_dtype=f64, out_transfer_dtype=f64))
            refs.append(O.truncate(O.add(A, C, 1.0, 0.5), mode="fixed", ranks=[r] * nn)[0])
        else:
            problems.append(dict(Xs=devs, coef=[1.0, 0.5], mode=H.HT_RANK_TOL, eps=1e-3, relative=True,
                                 precision=H.HT_PREC_FP64, out_frame_dtype=f64, out_transfer_dtype=f64))
            refs.append(O.truncate(O.add(A, C, 1.0, 0.5), mode="tol", eps=1e-3)[0])
    bt = H.BatchTruncator(problems)
    eager = [to_oracle(r.out) for r in bt()]
    torch.cuda.synchronize()
    again = [to_oracle(r.out) for r in bt()]
    spread = max(O.rel_diff(x, y) for x, y in zip(again, eager))
    worst = max(O.rel_diff(x, y) for x, y in zip(eager, refs))
    say(f"  eager vs oracle worst {worst:.3e}; two eager runs differ by {spread:.3e}")
    assert worst <= 1e-10
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        bt(stream=s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            bt(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in bt.outs:
            for u in o.leaves:
                u.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = [to_oracle(o) for o in bt.outs]
        e_eager = max(O.rel_diff(x, y) for x, y in zip(got, eager))
        e_or = max(O.rel_diff(x, y) for x, y in zip(got, refs))
        say(f"  replay {rep}: vs eager {e_eager:.3e}, vs oracle {e_or:.3e}")
        assert e_eager <= max(1e-13, 10 * spread) and e_or <= 1e-10
        bt()
        torch.cuda.synchronize()
