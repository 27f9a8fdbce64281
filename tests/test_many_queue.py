"""Host-side checks of the batched persistent launch's work queue (built by
the library's planner, no GPU): coverage of every transform, the ordering
that guarantees forward progress, and a simulated run of resident
workgroups pulling items from the queue under the kernel's wait rule."""
import numpy as np
import pytest

from paper_1707_07263_amd import capi, workloads

SINGLE, FIRST, SECOND = 0, 1, 2


def check_queue(sizes, schedule=None, threads=256, P=16):
    items, first_len, first_tiles = capi.fft_describe_many(list(sizes), capi.FFT_C64, schedule)
    sizes = np.asarray(sizes)
    lg = np.log2(sizes).astype(int)
    seen_first = {}
    first_done_pos = {}
    second_tiles = {}
    singles = np.zeros(len(sizes), int)
    for pos, (kind, tlg, a, b) in enumerate(items):
        if kind == FIRST:
            assert first_len[a] == (1 << tlg)
            seen_first.setdefault(a, set()).add(b)
            first_done_pos[a] = pos
            assert a not in second_tiles, "first-pass tile after a second-pass tile"
        elif kind == SECOND:
            # every first-pass tile of this transform precedes it in the queue
            assert len(seen_first.get(a, ())) == first_tiles[a]
            assert (1 << tlg) * first_len[a] == sizes[a]
            second_tiles.setdefault(a, set()).add(b)
        else:
            assert kind == SINGLE and b >= 1
            singles[a] += 0  # transform index of the tile's first line
    for i, n in enumerate(sizes):
        if first_tiles[i]:
            n1 = int(first_len[i])
            n2 = int(n) // n1
            assert n1 >= 2 and n2 >= 2
            # tiles cover the N2 columns of the first pass and N1 of the second
            assert seen_first[i] == set(range(first_tiles[i]))
            assert len(second_tiles[i]) >= 1 and second_tiles[i] == set(range(len(second_tiles[i])))
    n_single_lines = int(items[items[:, 0] == SINGLE][:, 3].sum())
    assert n_single_lines == int((first_tiles == 0).sum())
    return items, first_tiles


def simulate(items, first_tiles, workers, rng):
    """Workers take items in queue order; a second-pass item can finish only
    after all first-pass items of its transform finished.  Returns steps."""
    done = np.zeros(len(first_tiles), int)
    head = 0
    busy = []  # (remaining work, item)
    steps = 0
    while head < len(items) or busy:
        while len(busy) < workers and head < len(items):
            busy.append([int(rng.integers(1, 5)), items[head]])
            head += 1
        progressed = False
        for w in busy:
            kind, _, a, _ = w[1]
            if kind == SECOND and done[a] < first_tiles[a]:
                continue  # waiting
            w[0] -= 1
            progressed = True
        for w in [w for w in busy if w[0] <= 0]:
            if w[1][0] == FIRST:
                done[w[1][2]] += 1
            busy.remove(w)
        assert progressed, "deadlock: every resident worker waits"
        steps += 1
        assert steps < 10 * len(items) + 100
    return steps


def test_uneven_512_queue():
    sizes = workloads.uneven_sizes(512, 8, 16, seed=3)
    items, ft = check_queue(sizes)
    rng = np.random.default_rng(0)
    for workers in (1, 3, 64, 768):
        simulate(items, ft, workers, rng)


@pytest.mark.parametrize("schedule", [None, "pipe=0;threads=256;p=8", "pipe=0;threads=256;pass2=10",
                                      "pipe=0;threads=256;pass2=13;order=given", "pipe=0;threads=512",
                                      "pipe=0;threads=256;pass2=1", "pipe=0;threads=256;pass2=2;order=given",
                                      "pipe=0;threads=256;lag=1", "pipe=0;threads=256;lag=3;pass2=9",
                                      "pipe=0;threads=256;lag=100"])
def test_queue_all_lengths(schedule):
    g = np.random.default_rng(5)
    sizes = np.array([1 << e for e in list(range(0, 17)) * 2])
    g.shuffle(sizes)
    items, ft = check_queue(sizes, schedule)
    simulate(items, ft, 4, g)


def test_queue_large_lengths():
    sizes = [1 << 24, 1 << 20, 1 << 17, 8, 1]
    items, ft = check_queue(sizes)
    simulate(items, ft, 2, np.random.default_rng(1))


def test_queue_errors():
    for sizes, code in (([3], capi.FFT_ERR_UNSUPPORTED_SIZE), ([1 << 25], capi.FFT_ERR_UNSUPPORTED_SIZE)):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_describe_many(sizes)
        assert ei.value.status == code
    for bad in ("p=7", "threads=100", "pass2=0", "pass2=14", "order=random", "x=1", "lag=-1",
                "pipe=1;threads=256;pass2=13", "pipe=3", "pipe=2;threads=512;p=8", "ntail=-1", "ntst=2"):
        with pytest.raises(capi.FFTError) as ei:
            capi.fft_describe_many([256], schedule=bad)
        assert ei.value.status == capi.FFT_ERR_INVALID_ARGUMENT, bad


def test_queue_lag_interleaves():
    # with lag k the second-pass tiles of split transform i come right after
    # the first-pass tiles of transform i + k
    sizes = [1 << 20] * 6
    items, ft = check_queue(sizes, "pipe=0;threads=256;lag=2")
    kinds = [(int(k), int(a)) for k, _, a, _ in items]
    runs = []
    for k, a in kinds:
        if not runs or runs[-1] != (k, a):
            runs.append((k, a))
    assert runs == [(FIRST, 0), (FIRST, 1), (FIRST, 2), (SECOND, 0), (FIRST, 3), (SECOND, 1),
                    (FIRST, 4), (SECOND, 2), (FIRST, 5), (SECOND, 3), (SECOND, 4), (SECOND, 5)]
    for workers in (1, 2, 300):
        simulate(items, ft, workers, np.random.default_rng(workers))
    # lag 0 keeps every first-pass tile first
    items0, _ = check_queue(sizes)
    first = [i for i, it in enumerate(items0) if it[0] == FIRST]
    assert first == list(range(len(first)))


def simulate_ahead(items, first_tiles, workers, rng, ahead=1, static=True):
    """The pipelined kernel's protocol: worker w runs items w, w + workers,
    ... (static) or takes them from the queue `ahead` beyond the one it runs
    (dynamic), in order; it releases a finished first-pass item only after
    it has started its next item (or before any wait, or at exit), and a
    second-pass item starts only after every first-pass item of its
    transform is released."""
    done = np.zeros(len(first_tiles), int)
    head = 0
    held = [[] for _ in range(workers)]     # items taken, in order
    left = [None] * workers
    pending = [None] * workers
    steps = 0

    nexts = list(range(workers))

    def take(w):
        nonlocal head
        while len(held[w]) < 1 + ahead:
            if static:
                if nexts[w] >= len(items):
                    return
                held[w].append(items[nexts[w]])
                nexts[w] += workers
            else:
                if head >= len(items):
                    return
                held[w].append(items[head])
                head += 1

    for w in range(workers):
        take(w)
    while any(held):
        progressed = False
        for w in range(workers):
            if not held[w]:
                if pending[w] is not None:
                    done[pending[w]] += 1
                    pending[w] = None
                    progressed = True
                continue
            kind, _, a, _ = held[w][0]
            if left[w] is None:
                if kind == SECOND and done[a] < first_tiles[a]:
                    if pending[w] is not None:   # release before waiting
                        done[pending[w]] += 1
                        pending[w] = None
                        progressed = True
                    continue
                left[w] = int(rng.integers(1, 5))
                if pending[w] is not None:       # released mid-way through the next item
                    done[pending[w]] += 1
                    pending[w] = None
            left[w] -= 1
            progressed = True
            if left[w] == 0:
                left[w] = None
                held[w].pop(0)
                if kind == FIRST:
                    pending[w] = a
                take(w)
        assert progressed, "deadlock: every worker waits"
        steps += 1
    assert (done == first_tiles).all()
    return steps


@pytest.mark.parametrize("schedule", ["pipe=1;threads=512", "pipe=1;threads=512;pass2=1",
                                      "pipe=1;threads=512;lag=2", "pipe=1;threads=512;order=given",
                                      "pipe=1;threads=256", "pipe=1;threads=256;pass2=5"])
def test_queue_pipelined_protocol(schedule):
    sizes = workloads.uneven_sizes(512, 8, 16, seed=3)
    items, ft = check_queue(sizes, schedule)
    for workers in (1, 2, 7, 256, 3000):
        simulate_ahead(items, ft, workers, np.random.default_rng(workers))
        simulate_ahead(items, ft, workers, np.random.default_rng(workers), ahead=2, static=False)
    # uniform large transforms: every second-pass item depends on tiles taken
    # by many workers
    items, ft = check_queue([1 << 16] * 64, "pipe=1;threads=512")
    for workers in (1, 3, 256):
        simulate_ahead(items, ft, workers, np.random.default_rng(5 + workers))


@pytest.mark.parametrize("schedule", ["pipe=2;threads=512", "pipe=2;threads=512;pass2=9",
                                      "pipe=2;threads=512;pass.12=2;n1.16=6;n1.15=9"])
def test_two_launch_split(schedule):
    # the two-launch kernel: launch 0 holds every first-pass and one-pass
    # tile, launch 1 every second-pass tile; every transform is covered
    sizes = workloads.uneven_sizes(512, 8, 16, seed=3)
    items, first_len, first_tiles = capi.fft_describe_many(list(sizes), capi.FFT_C64, schedule)
    q = capi.fft_describe_many_launches(list(sizes), capi.FFT_C64, schedule)
    assert len(q) == 3 and q[0] == 0 and q[2] == len(items)
    l0, l1 = items[q[0]:q[1]], items[q[1]:q[2]]
    assert np.all(l0[:, 0] != SECOND) and np.all(l1[:, 0] == SECOND)
    check_queue(sizes, schedule)
    split = {int(a) for a in np.nonzero(first_tiles)[0]}
    assert {int(a) for a in l1[:, 2]} == split
    # the per-length choices took effect
    lg = np.log2(sizes).astype(int)
    if "n1.16=6" in schedule:
        assert np.all(first_len[lg == 16] == 64) and np.all(first_len[lg == 15] == 512)
    if "pass.12=2" in schedule:
        assert np.all(first_tiles[lg == 12] > 0)


def simulate_two_launch(n_items, workers, rng):
    """One launch of the two-launch kernel: worker g starts with items g and
    workers + g, then claim k (in the order the claims reach the queue head)
    names item 2 * workers + k; an index past the end stops the worker.
    Returns how many times each item ran."""
    ran = np.zeros(n_items, int)
    head = 0
    cur = [g if g < n_items else None for g in range(workers)]
    nxt = [workers + g if workers + g < n_items else None for g in range(workers)]
    live = [g for g in range(workers) if cur[g] is not None]
    while live:
        g = live[int(rng.integers(len(live)))]
        ran[cur[g]] += 1
        cur[g] = nxt[g]
        nxt[g] = None
        if cur[g] is not None:
            k = head
            head += 1
            if 2 * workers + k < n_items:
                nxt[g] = 2 * workers + k
        else:
            live.remove(g)
    return ran


@pytest.mark.parametrize("n_items,workers", [(846, 256), (854, 256), (1, 256), (255, 256), (256, 256),
                                             (511, 256), (512, 256), (513, 256), (100, 1), (100, 7)])
def test_two_launch_static_first_items(n_items, workers):
    # every item of a launch runs exactly once under the fixed first two
    # items and the dynamic claims after them, whatever order workers finish in
    for seed in range(3):
        ran = simulate_two_launch(n_items, workers, np.random.default_rng(seed))
        assert np.all(ran == 1)


def two_launch_counts(n_items, workers, first_claim_at_entry, rng):
    """Items per worker when every item takes one time unit: worker g starts
    at a jittered time, issues its first claim at kernel entry (or once its
    first item's loads are in, one unit later), and each later claim at the
    top of an iteration; claims are served in the order they are issued."""
    start = rng.uniform(0.0, 0.2, workers)
    first = start if first_claim_at_entry else start + rng.uniform(0.0, 1.5, workers)
    count = np.zeros(workers, int)
    for g in range(workers):
        count[g] = int(g < n_items) + int(workers + g < n_items)
    events = sorted((first[g], g) for g in range(workers))
    head = 0
    pending = []
    # a worker's k-th top comes at start + k; a claim issued at its top j
    # (j >= 0) is issued at start + j, the entry claim at `first`
    for t, g in events:
        pending.append((t, g))
    for g in range(workers):
        for j in range(n_items):
            pending.append((start[g] + 1.0 + j, g))
    pending.sort()
    alive = count > 1
    for t, g in pending:
        if not alive[g]:
            continue
        idx = 2 * workers + head
        head += 1
        if idx < n_items:
            count[g] += 1
        else:
            alive[g] = False
    return count


@pytest.mark.parametrize("n_items", [768, 846, 854])
def test_two_launch_first_claim_at_entry(n_items):
    # with the first claim issued at kernel entry every first claim is
    # served before any second one, so equal items split evenly (3 or 4 for
    # 846 items on 256 workgroups); a first claim issued after the first
    # item's loads can lose to other workgroups' second claims
    rng = np.random.default_rng(11)
    even = two_launch_counts(n_items, 256, True, rng)
    assert even.sum() == n_items
    assert even.max() - even.min() <= 1, (even.min(), even.max())
    late = two_launch_counts(n_items, 256, False, rng)
    assert late.sum() == n_items


def test_per_length_schedule_items():
    sizes = [1 << 14, 1 << 9, 1 << 16]
    _, fl, ft = capi.fft_describe_many(sizes, capi.FFT_C64, "n1.14=5;pass.9=2;n1.16=12")
    assert list(fl) == [32, 32, 4096] and all(ft > 0)
    _, fl, ft = capi.fft_describe_many(sizes + [1 << 12], capi.FFT_C64, "pass.12=2;pass.9=1")
    assert fl[3] == 64 and ft[3] > 0 and fl[1] == 0
    _, fl, ft = capi.fft_describe_many(sizes + [1 << 12], capi.FFT_C64, "pass2=9;pass.12=1")
    assert fl[3] == 0 and ft[3] == 0 and fl[1] > 0
    for bad in ("n1.16=13", "n1.16=3", "pass.13=1", "pass.9=3", "n1.0=1", "n1.x=2", "nx.9=2"):
        with pytest.raises(capi.FFTError):
            capi.fft_describe_many(sizes + [1 << 15, 1 << 13], capi.FFT_C64, bad)
    assert len(capi.fft_describe_many_launches(sizes, capi.FFT_C64, None)) == 3  # default: two launches
    assert len(capi.fft_describe_many_launches(sizes, capi.FFT_C64, "pipe=0;threads=256")) == 2
