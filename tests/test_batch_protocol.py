"""CPU checks of the batched form's work-item table and of the one-launch
protocol, on the library's own descriptor layout (dft3d_batch_describe, the
same layout code the batched call uploads).

The persistent kernel hands out tickets (tile numbers in level-major order)
from a counter; a tile of pass k of a problem first waits until every tile of
pass k - 1 of that problem is counted done.  The launch drains for any
number of resident workgroups exactly when every item's dependency lies
entirely at smaller tickets and its done-count target equals the number of
tiles that count it.  These tests check both on the real tables and then run
the protocol itself with emulated workgroups (one, a few, many; random
completion orders), including the counters the last workgroup zeroes for
the next launch, and a planted bad table (on the CPU only) that must end in
the error flag instead of a hang."""
import math
import random

import pytest

from paper_1904_10119_amd import dft3d, inputs

SMALL_MIX = [(32, 64, 128), (128, 32, 64), (64, 64, 64), (8, 16, 4), (2, 2, 2),
             (1, 1, 1), (32, 32, 32), (128, 128, 16)]
BATCHES = {
    "small mix": SMALL_MIX,
    "96 seed 104": inputs.batch_shapes(96, 104),
    "96 seed 7": inputs.batch_shapes(96, 7),
    "planes": [(2, a, b) for a in (32, 64, 128) for b in (32, 64, 128)] + [(4, 16, 64)],
}


def tables():
    for name, shapes in BATCHES.items():
        for schedule in ("pencil", "slab", "auto"):
            for launch in ("levels", "persistent"):
                yield name, shapes, schedule, launch


def find_item(items, ticket):
    """The kernel's binary search: last item whose first tile <= ticket."""
    lo, hi = 0, len(items) - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if items[mid]["first"] <= ticket:
            lo = mid
        else:
            hi = mid - 1
    return lo


def pass_count(shape, schedule, launch):
    """Passes of one problem as the batched call runs it: the plan's own, or
    for fused plane passes the form does not cover, the unfused plan's."""
    d = dft3d.describe(shape, schedule)
    for p in d["passes"]:
        if "plane" in p["label"] or p.get("plane_rows", 0):
            n1, n2 = shape[1], shape[2]
            ok = n1 in (32, 64, 128) and n2 in (32, 64, 128)
            if launch == "persistent":
                ok = ok and n1 * n2 <= 4096
            if not ok:
                return len(dft3d.describe(shape, schedule, fused_plane=0)["passes"])
    return len(d["passes"])


@pytest.mark.parametrize("name,shapes,schedule,launch", list(tables()))
def test_item_table_is_consistent(name, shapes, schedule, launch):
    d = dft3d.describe_batch(shapes, schedule, launch)
    assert d["batchable"], (name, schedule)
    items = d["items"]
    assert d["total"] == sum(it["ntiles"] for it in items)
    # tickets: consecutive ranges in item order, covering [0, total)
    nxt = 0
    for it in items:
        assert it["first"] == nxt
        assert it["ntiles"] >= 1
        nxt += it["ntiles"]
    # tiles cover every pencil (plane) of the pass exactly
    for it in items:
        if it["n1"]:
            assert it["ntiles"] == it["pencils"]
            if launch == "persistent":
                assert it["n1"] * it["n"] <= 4096
        else:
            assert it["ntiles"] == math.ceil(it["pencils"] / it["tile"])
            assert it["n"] <= 256 and it["tile"] * (it["n"] // max(1, it["n"])) >= 1
    # every problem: passes 0..k-1 in order, each waiting for the previous
    by_problem = {}
    for k, it in enumerate(items):
        by_problem.setdefault(it["problem"], []).append(k)
    assert sorted(by_problem) == list(range(len(shapes)))
    for prob, ks in by_problem.items():
        assert [items[k]["pass"] for k in ks] == list(range(len(ks)))
        assert len(ks) == pass_count(shapes[prob], schedule, launch), (prob, shapes[prob])
        assert items[ks[0]]["dep"] == -1
        for a, b in zip(ks, ks[1:]):
            assert items[b]["dep"] == a
            # the whole dependency lies at smaller tickets
            assert items[a]["first"] + items[a]["ntiles"] <= items[b]["first"]
    # the binary search maps every ticket to the item that owns it
    for t in sorted({0, d["total"] - 1} | {it["first"] for it in items} |
                    {it["first"] + it["ntiles"] - 1 for it in items}):
        k = find_item(items, t)
        assert items[k]["first"] <= t < items[k]["first"] + items[k]["ntiles"]
    if launch == "persistent":
        assert d["threads"] == 256
        # at least one workgroup fits a CU's 160 KiB of LDS (the protocol
        # itself needs no co-residency: see the one-workgroup emulation)
        assert d["lds_bytes"] <= 160 * 1024
    else:
        # level launches: each level is a contiguous ticket range of one kind
        for L in d["levels"]:
            its = items[L["item_lo"]:L["item_hi"]]
            assert its[0]["first"] == L["base"]
            assert sum(i["ntiles"] for i in its) == L["ntiles"]


class Emulator:
    """The persistent kernel's ticket / wait / count protocol with W
    emulated workgroups.  Each step advances one workgroup chosen at random:
    take a ticket, poll its dependency (bounded by spin_limit polls), run
    the tile (a random number of steps), count it done, and on leaving let
    the last workgroup zero the counters."""

    def __init__(self, items, total, workers, rng, spin_limit=10**9):
        self.items, self.total, self.W, self.rng = items, total, workers, rng
        self.spin_limit = spin_limit
        self.head = 0
        self.exited = 0
        self.error = 0
        self.done = [0] * len(items)

    def launch(self):
        items = self.items
        ran = {}
        # per workgroup: state, ticket, item, polls, remaining work
        wg = [{"st": "take"} for _ in range(self.W)]
        live = set(range(self.W))
        steps = 0
        while live:
            steps += 1
            assert steps < 50 * (self.total + 10) * max(1, self.W) + 10**6, "no progress"
            w = self.rng.choice(sorted(live))
            s = wg[w]
            if s["st"] == "take":
                t = self.head
                self.head += 1
                if t >= self.total:
                    live.discard(w)
                    self.exited += 1
                    if self.exited == self.W:  # last one out zeroes the counters
                        self.done = [0] * len(items)
                        self.head = 0
                        self.exited = 0
                    continue
                k = find_item(items, t)
                s.update(st="wait", t=t, k=k, polls=0)
            if s["st"] == "wait":
                dep = items[s["k"]]["dep"]
                if dep >= 0 and self.done[dep] < items[dep]["ntiles"]:
                    s["polls"] += 1
                    if s["polls"] >= self.spin_limit or (s["polls"] % 64 == 0 and self.error):
                        self.error = 1
                    else:
                        continue
                if dep >= 0 and not self.error:
                    # the dependency is complete when the tile starts
                    assert self.done[dep] == items[dep]["ntiles"]
                s.update(st="run", left=self.rng.randint(0, 3))
                continue
            if s["st"] == "run":
                if s["left"] > 0:
                    s["left"] -= 1
                    continue
                key = (s["k"], s["t"] - items[s["k"]]["first"])
                ran[key] = ran.get(key, 0) + 1
                self.done[s["k"]] += 1
                s.update(st="take")
        return ran


@pytest.mark.parametrize("name", ["small mix", "96 seed 104"])
@pytest.mark.parametrize("schedule", ["pencil", "slab"])
@pytest.mark.parametrize("workers", [1, 2, 7, 64])
def test_persistent_protocol_drains(name, schedule, workers):
    shapes = BATCHES[name]
    d = dft3d.describe_batch(shapes, schedule, "persistent")
    items, total = d["items"], d["total"]
    rng = random.Random(1000 * workers + len(shapes))
    em = Emulator(items, total, workers, rng)
    for launch in range(2):  # a second launch starts from the zeroed counters
        assert em.head == 0 and em.exited == 0 and not any(em.done)
        ran = em.launch()
        assert em.error == 0
        assert len(ran) == total and all(v == 1 for v in ran.values())
        for k, it in enumerate(items):
            for tile in range(it["ntiles"]):
                assert (k, tile) in ran


def test_planted_forward_dependency_ends_in_error_not_hang():
    """A table whose dependency points at a later item (planted here, on the
    CPU) can never be satisfied by one workgroup: the bounded wait must give
    up, flag the error, and the launch must still drain."""
    d = dft3d.describe_batch(SMALL_MIX, "pencil", "persistent")
    items = [dict(it) for it in d["items"]]
    # make the first level-0 item wait for the last item
    items[0]["dep"] = len(items) - 1
    em = Emulator(items, d["total"], 1, random.Random(5), spin_limit=50)
    ran = em.launch()
    assert em.error == 1
    assert len(ran) == d["total"]


def test_describe_batch_rejects_bad_arguments():
    import ctypes
    L = dft3d.lib()
    arr = (ctypes.c_int64 * 3)(4, 4, 4)
    assert L.dft3d_batch_describe(arr, -1, 2, 0, None, 0, None) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_batch_describe(None, 1, 2, 0, None, 0, None) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_batch_describe(arr, 1, 2, 2, None, 0, None) == dft3d.ERR_INVALID_ARG
    bad = (ctypes.c_int64 * 3)(4, 0, 4)
    assert L.dft3d_batch_describe(bad, 1, 2, 0, None, 0, None) == dft3d.ERR_UNSUPPORTED_SIZE
    assert L.dft3d_batch_describe(arr, 0, 2, 1, None, 0, None) == dft3d.OK


def test_long_axes_and_split_axes_not_batchable():
    """Passes longer than 256 and four-step passes (volumetric) are not
    batched items: such batches run plan by plan."""
    d = dft3d.describe_batch([(1024, 4, 8), (16, 16, 16)], "pencil", "persistent")
    assert not d["batchable"]
    d = dft3d.describe_batch([(64, 64, 64)], "volumetric", "levels")
    assert not d["batchable"]
