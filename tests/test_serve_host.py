"""Host logic of the server (no GPU): admission by slots and HBM footprint."""


def _admission():
    # importing the package loads no GPU state; Admission is plain host logic
    import paper_2408_10982_amd.serve as S
    return S.Admission


def test_admission_slots_and_budget():
    Admission = _admission()
    a = Admission(slots=2, budget=100)
    for j, fp in enumerate([60, 30, 50, 10]):
        a.push(j, fp)
    assert a.pop() == (0, 60)
    assert a.pop() == (1, 30)          # 90 <= 100
    assert a.pop() is None             # slots full
    a.release(60)
    assert a.pop() == (2, 50)          # 30 + 50 <= 100
    assert a.pop() is None             # slots full again
    a.release(30)
    a.release(50)
    assert a.pop() == (3, 10)
    assert a.max_in_flight == 2


def test_admission_refuses_over_budget_and_keeps_order():
    Admission = _admission()
    a = Admission(slots=8, budget=100)
    a.push("big", 90)
    a.push("small", 5)
    a.push("huge", 500)
    assert a.pop() == ("big", 90)
    assert a.pop() == ("small", 5)
    assert a.pop() is None             # 500 does not fit beside 95
    a.release(90)
    assert a.pop() is None             # still not beside 5
    a.release(5)
    assert a.pop() == ("huge", 500)    # alone it is admitted
    assert a.in_flight == 1 and a.reserved == 500


def test_admission_counts_resident_bytes():
    """Resident bytes (pools, workspaces) come off the budget before the
    in-flight queries' footprints; the first query is admitted regardless."""
    A = _admission()(slots=4, budget=100)
    for j in range(3):
        A.push(j, 30)
    assert A.pop(held=60)[0] == 0          # alone: admitted whatever it needs
    assert A.pop(held=60) is None          # 60 + 30 + 30 > 100
    assert A.pop(held=30)[0] == 1          # 30 + 30 + 30 <= 100
    assert A.pop(held=30) is None


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and
    says so, before any GPU work."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and "--gpus 2" in r.stderr
