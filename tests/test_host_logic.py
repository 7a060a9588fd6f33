"""The host runtime's pure logic (sfhk_host.hpp: birth order of the samples and tiles, unfinished
tiles, the longest-first work list of several jobs and its kernel segments, duplicate handles, the
checkpoint layout and header check, the spectrum's work plan), compiled for the host with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and checked against plain Python
statements of what each must compute, on random and edge cases. The library calls the same
header (CPU only, no GPU)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "host_logic_driver.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("host") / "host_logic")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Werror",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe, DRIVER],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

    def call(lines):
        r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                           timeout=300, env=env)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
        out = r.stdout.splitlines()
        assert len(out) == len(lines)
        return out
    return call


def _ints(s):
    return [int(x) for x in s.split()]


# ------------------------------------------------------------------------------------------
def _sort_case(rng, n, ns, tile, ordered):
    n0 = rng.integers(0, ns + 1, n)
    if ordered:
        n0 = np.sort(n0)
    npad = (n + tile - 1) // tile * tile if n else 0
    return n0, npad


def test_birth_order_is_the_stable_sort_by_birth_step(run):
    rng = np.random.default_rng(11)
    cases = []
    for k in range(300):
        n = int(rng.choice([0, 1, 63, 64, 65, 130, int(rng.integers(1, 2000))]))
        ns = int(rng.choice([0, 1, 7, int(rng.integers(1, 5000))]))
        cases.append((*_sort_case(rng, n, ns, 64, k % 3 == 0), ns))
    out = run([f"sort {len(n0)} {ns} {npad} 64 " + " ".join(map(str, n0)) for n0, npad, ns in cases])
    for (n0, npad, ns), line in zip(cases, out):
        assert line.startswith("ok")
        perm, n0s, tn0, nxt, last = (_ints(x) for x in line[2:].split("|"))
        want = list(np.argsort(n0, kind="stable")) + [-1] * (npad - len(n0))
        assert perm == want
        assert n0s == [int(n0[i]) for i in want[:len(n0)]] + [ns + 1] * (npad - len(n0))
        assert tn0 == n0s[::64] and nxt == tn0 and last == [t - 1 for t in tn0]
        assert all(a <= b for a, b in zip(n0s, n0s[1:]))


def test_birth_steps_out_of_range_are_refused(run):
    out = run(["sort 3 10 64 64 0 11 2", "sort 2 10 64 64 -1 0", "sort 3 10 2 64 0 1 2",
               "sort 1 10 64 64 10"])
    assert out[:3] == ["bad"] * 3 and out[3].startswith("ok")


def test_unfinished_tiles_are_the_prefix_with_steps_left(run):
    rng = np.random.default_rng(12)
    lines, want = [], []
    for _ in range(400):
        ns = int(rng.integers(0, 3000))
        tn0 = np.sort(rng.integers(0, ns + 2, int(rng.integers(0, 50))))
        done = int(rng.choice([0, 1, ns, ns + 1, int(rng.integers(0, 2 * ns + 2))]))
        lines.append(f"unfinished {ns} {done} {len(tn0)} " + " ".join(map(str, tn0)))
        want.append(int(np.sum(tn0 + done <= ns)))
    assert [int(x) for x in run(lines)] == want


def _work_ref(jobs, nsegs):
    items = []
    for i, (ns, sd, done, seg, tn0) in enumerate(jobs):
        if done:
            continue
        nt = sum(1 for a in tn0 if a + sd <= ns)
        items += [(ns + 1 - (tn0[t] + sd), i, t, seg) for t in range(nt)]
    items.sort(key=lambda x: (x[3], -x[0]))  # Python's sort is stable
    n_items = [sum(1 for x in items if x[3] == g) for g in range(nsegs)]
    offset = [int(v) for v in np.concatenate([[0], np.cumsum(n_items)[:-1]])]
    return items, n_items, offset


def test_work_list_is_longest_first_per_segment(run):
    rng = np.random.default_rng(13)
    cases, lines = [], []
    for _ in range(150):
        nj, nsegs = int(rng.integers(0, 12)), 8
        jobs = []
        for _ in range(nj):
            ns = int(rng.integers(1, 4000))
            tn0 = sorted(int(x) for x in rng.integers(0, ns + 1, int(rng.integers(0, 40))))
            sd = int(rng.choice([0, int(rng.integers(0, ns + 2))]))
            jobs.append((ns, sd, int(rng.random() < 0.15), int(rng.integers(0, nsegs)), tn0))
        cases.append((jobs, nsegs))
        lines.append(f"work {nj} {nsegs} " + " ".join(
            f"{ns} {sd} {d} {seg} {len(t)} " + " ".join(map(str, t)) for ns, sd, d, seg, t in jobs))
    for (jobs, nsegs), line in zip(cases, run(lines)):
        items_s, n_s, off_s = line[len("items"):].split("|")
        v = _ints(items_s)
        got = [tuple(v[k:k + 4]) for k in range(0, len(v), 4)]
        items, n_items, offset = _work_ref(jobs, nsegs)
        assert got == items
        assert _ints(n_s) == n_items and _ints(off_s) == offset


def test_duplicate_handles(run):
    rng = np.random.default_rng(14)
    lines, want = [], []
    for _ in range(200):
        n = int(rng.integers(0, 30))
        v = rng.integers(1, 40, n)
        lines.append(f"dup {n} " + " ".join(map(str, v)))
        want.append(int(len(set(v.tolist())) != n))
    assert [int(x) for x in run(lines)] == want


def _hdr(magic=1, n_traj=100, n_pad=128, n_tiles=2, n_steps=50, acc=6936, sd=10, kind=1, prec=0,
         done=0, fp=12345678901234567):
    return f"{magic} {n_traj} {n_pad} {n_tiles} {n_steps} {acc} {sd} {kind} {prec} {done} {fp}"


def test_checkpoint_layout_and_header_check(run):
    rng = np.random.default_rng(15)
    lines, want = [], []
    for _ in range(100):
        b = [int(x) for x in rng.integers(0, 10 ** 7, int(rng.integers(0, 12)))]
        lines.append(f"ckpt {len(b)} " + " ".join(map(str, b)) + f" | {_hdr()} | {_hdr()}")
        off, o = [], 256
        for x in b:
            off.append(o)
            o += (x + 255) // 256 * 256
        want.append((off, o))
    for line, (off, total) in zip(run(lines), want):
        layout, match = line.split("|")
        assert _ints(layout) == off + [total] and int(match) == 1
    job = _hdr()
    bad = [_hdr(magic=0), _hdr(n_traj=101), _hdr(n_pad=192), _hdr(n_tiles=3), _hdr(n_steps=51),
           _hdr(acc=13872), _hdr(sd=-1), _hdr(kind=2), _hdr(prec=1), _hdr(done=2),
           _hdr(fp=12345678901234568)]
    good = [_hdr(sd=0), _hdr(sd=51, done=1)]
    out = run([f"ckpt 0 | {h} | {job}" for h in bad + good])
    assert [int(x.split("|")[1]) for x in out] == [0] * len(bad) + [1] * len(good)


def test_spectrum_plan(run):
    lines, cases = [], []
    for n, nfft in [(1, 1), (2208, 2208), (2208, 4416), (32768, 32768), (32768, 65536),
                    (65536, 65536), (1023, 2048), (1025, 2048), (64 * 1024 + 1, 1 << 17),
                    (3_000_000, 1 << 22)]:
        lines.append(f"plan {n} {nfft} 1024 64")
        cases.append((n, nfft))
    for (n, nfft), line in zip(cases, run(lines)):
        nk, span, nsp, xw, tw, part, tot = _ints(line)
        chunks = -(-n // 1024)
        assert nk == nfft // 2 + 1
        assert span % 1024 == 0 and span * nsp >= n and span * (nsp - 1) < n and nsp <= 64
        assert span == -(-chunks // 64) * 1024
        a = lambda b: -(-b // 256) * 256
        assert (xw, tw, part) == (0, a(8 * nfft), a(8 * nfft) + a(16 * nfft))
        assert tot == part + a(16 * nsp * nk)
