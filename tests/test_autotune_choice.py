"""Host logic of the autotuner's choice (no GPU): the fastest candidate wins, except that hardware
dispatch is kept against a persistent form that is not faster by the stated margin."""
from paper_2601_17164_amd import autotune as A


def test_fastest_hardware_dispatch_wins():
    r = {"workers=0,chunk=0": 10.0, "workers=0,chunk=2048": 9.0, "workers=4,chunk=0": 8.0}
    assert A.choose(r) == "workers=0,chunk=0"


def test_near_tie_keeps_hardware_dispatch():
    r = {"workers=0,chunk=0": 10.0, "workers=0,chunk=2048": 9.0, "workers=4,chunk=0": 10.2}
    assert A.choose(r) == "workers=0,chunk=0"


def test_clear_persistent_win_is_taken():
    r = {"workers=0,chunk=0": 10.0, "workers=8,chunk=2048": 10.0 * A.PERSISTENT_MARGIN * 1.01}
    assert A.choose(r) == "workers=8,chunk=2048"


def test_without_hardware_candidates_the_fastest_wins():
    r = {"workers=4,chunk=0": 3.0, "workers=16,chunk=0": 4.0}
    assert A.choose(r) == "workers=16,chunk=0"


def test_candidate_forms_cover_workers_and_chunks():
    forms = A.forms()
    assert len(forms) == len(A.WORKERS) * len(A.CHUNKS) == len(set(forms))
    assert {A.parse(f) for f in forms} == {(w, k) for w in A.WORKERS for k in A.CHUNKS}
    assert 0 in A.WORKERS and 0 in A.CHUNKS and min(k for k in A.CHUNKS if k) <= 256


def test_finalists_are_each_worker_counts_best_chunk():
    r = {"workers=0,chunk=0": 10.0, "workers=0,chunk=256": 7.0, "workers=8,chunk=256": 6.0,
         "workers=8,chunk=4096": 9.5, "workers=16,chunk=0": 9.0}
    assert A.finalists(r) == ["workers=0,chunk=0", "workers=8,chunk=4096", "workers=16,chunk=0"]


def test_second_stage_takes_the_fastest_without_margin():
    r = {"workers=0,chunk=0": 10.0, "workers=8,chunk=0": 10.01}
    assert A.choose(r, margin=1.0) == "workers=8,chunk=0"
    assert A.choose(r) == "workers=0,chunk=0"
