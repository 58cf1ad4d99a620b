"""The persistent batched schedule on the CPU: its claim order (host code of
the library), a model of the schedule that shows it completes whatever the
number of resident workgroups, and the memory scopes of its device
synchronisation as the compiler emitted them for gfx950.

The model: a workgroup is resident from its start until it leaves; at most
`slots` are resident, and the rest start, in index order, as slots free up.
A resident workgroup either takes its next work item or runs the one it
holds once the pass before it (in its circuit's chain) has finished.  With
items handed out from one counter in the claim order, only running
workgroups hold items, and the smallest unfinished item always has its
dependency finished, so the run completes for any number of slots.  With
items bound to workgroup indices instead (item k to workgroup k mod G), a
grid larger than what is resident can leave every resident workgroup
waiting on an item held by one that has not started."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2602_09020_amd import cfh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm/bin"


def random_batch(rng, count):
    chain_len = rng.integers(1, 12, size=count)
    pass_items = rng.integers(1, 7, size=int(chain_len.sum()))
    amps = 2.0 ** rng.integers(12, 21, size=count)
    return chain_len, pass_items, amps


def chains_of(chain_len):
    out, p = [], 0
    for L in chain_len:
        out.append(list(range(p, p + int(L))))
        p += int(L)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_claim_order_is_a_permutation_that_respects_every_chain(seed):
    rng = np.random.default_rng(seed)
    chain_len, pass_items, amps = random_batch(rng, int(rng.integers(1, 40)))
    tp, ti, prev = cfh.cfh_batch_order(chain_len, pass_items, amps)
    chains = chains_of(chain_len)
    # every work item exactly once
    got = sorted(zip(tp.tolist(), ti.tolist()))
    want = sorted((p, i) for p in range(len(pass_items)) for i in range(pass_items[p]))
    assert got == want
    # prev is the pass before in the chain
    for ch in chains:
        assert prev[ch[0]] == -1
        for a, b in zip(ch, ch[1:]):
            assert prev[b] == a
    # every item after all items of the pass before it
    last = {}
    first = {}
    for k, p in enumerate(tp.tolist()):
        last[p] = k
        first.setdefault(p, k)
    for p in range(len(pass_items)):
        if prev[p] >= 0:
            assert first[p] > last[prev[p]]
    # level by level: pass lv of every chain before pass lv + 1 of any
    level = {p: lv for ch in chains for lv, p in enumerate(ch)}
    lv_seq = [level[p] for p in tp.tolist()]
    assert lv_seq == sorted(lv_seq)
    # within a level, the circuit with the most work left first
    circ = {p: c for c, ch in enumerate(chains) for p in ch}
    for lv in set(lv_seq):
        order = []
        for p in tp.tolist():
            if level[p] == lv and (not order or order[-1] != circ[p]):
                order.append(circ[p])
        left = [amps[c] * (chain_len[c] - lv) for c in order]
        assert left == sorted(left, reverse=True)


def test_claim_order_rejects_bad_sizes():
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_batch_order([2], [1, 0], [4096.0])
    assert e.value.code == cfh.CFH_E_INVAL
    with pytest.raises(cfh.CfhError) as e:
        cfh.cfh_batch_order([-1], [], [4096.0])
    assert e.value.code == cfh.CFH_E_INVAL


def run_model(tp, prev, pass_items, slots, grid, rng, bound):
    """Simulate the schedule; True if every item finishes, False on deadlock.
    bound = False: items from one counter in claim order; True: item k belongs
    to workgroup k mod grid, taken in order."""
    nt = len(tp)
    done = np.zeros(len(pass_items), np.int64)
    ready = np.zeros(len(pass_items), bool)
    next_ticket = 0
    own = [list(range(w, nt, grid)) for w in range(grid)] if bound else None
    held = {}          # workgroup -> ticket it holds
    resident = []
    started = 0
    finished_items = 0
    while finished_items < nt:
        while len(resident) < slots and started < grid:
            resident.append(started)
            started += 1
        movable = []
        for w in resident:
            if w in held:
                p = tp[held[w]]
                if prev[p] < 0 or ready[prev[p]]:
                    movable.append(w)
            else:
                movable.append(w)   # claims next, or leaves
        if not movable:
            return False
        w = movable[rng.integers(len(movable))]
        if w in held:
            p = tp[held.pop(w)]
            done[p] += 1
            finished_items += 1
            if done[p] == pass_items[p]:
                ready[p] = True
        elif bound:
            if own[w]:
                held[w] = own[w].pop(0)
            else:
                resident.remove(w)
        else:
            if next_ticket < nt:
                held[w] = next_ticket
                next_ticket += 1
            else:
                resident.remove(w)
    return True


@pytest.mark.parametrize("seed", range(4))
def test_model_counter_schedule_completes_for_any_residency(seed):
    rng = np.random.default_rng(100 + seed)
    chain_len, pass_items, amps = random_batch(rng, 25)
    tp, ti, prev = cfh.cfh_batch_order(chain_len, pass_items, amps)
    for slots in (1, 2, 5, 64):
        for grid in (slots, 4 * slots, 1000):
            assert run_model(tp, prev, pass_items, slots, grid, rng, bound=False), (slots, grid)


def test_model_index_bound_schedule_can_deadlock_beyond_residency():
    hits = 0
    for seed in range(20):
        rng = np.random.default_rng(200 + seed)
        chain_len, pass_items, amps = random_batch(rng, 25)
        tp, ti, prev = cfh.cfh_batch_order(chain_len, pass_items, amps)
        # a grid that fits: every workgroup resident, no deadlock
        assert run_model(tp, prev, pass_items, 16, 16, rng, bound=True)
        # a grid beyond residency
        hits += not run_model(tp, prev, pass_items, 4, 16, rng, bound=True)
    assert hits > 0


def _device_code(obj, tmp):
    fat = os.path.join(tmp, "b.fatbin")
    dev = os.path.join(tmp, "b.gfx950.o")
    subprocess.run([f"{LLVM}/llvm-objcopy", "--dump-section", f".hip_fatbin={fat}", obj, os.path.join(tmp, "h.o")],
                   check=True, capture_output=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fat}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={dev}"], check=True, capture_output=True)
    return subprocess.run([f"{LLVM}/llvm-objdump", "-d", "--no-show-raw-insn", dev], check=True,
                          capture_output=True, text=True).stdout


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "paper_2602_09020_amd", "_build", "batch2.o"))
                    or not os.path.exists(f"{LLVM}/llvm-objdump"),
                    reason="library objects or ROCm LLVM tools not present")
def test_persistent_kernel_synchronises_at_device_scope(tmp_path):
    """In every built persistent kernel: the dependency polls (the loop with
    s_sleep) read with sc1, so they bypass the XCD's own L2 and see a store
    made on any XCD; stores are written back past that L2 (buffer_wbl2 sc1)
    before an item is counted or a pass marked ready; and the caches are
    invalidated (buffer_inv sc1) before an item reads what others wrote."""
    dis = _device_code(os.path.join(ROOT, "paper_2602_09020_amd", "_build", "batch2.o"), str(tmp_path))
    kernels = re.split(r"\n(?=[0-9a-f]+ <)", dis)
    persist = [k for k in kernels if "k_batch_persist" in k.split("\n", 1)[0]]
    assert len(persist) == 12
    for k in persist:
        lines = [l.split("//")[0].strip() for l in k.split("\n")]
        sleeps = [i for i, l in enumerate(lines) if l.startswith("s_sleep")]
        assert sleeps
        for i in sleeps:
            window = [l for l in lines[i - 40:i + 12] if l.startswith("global_load")]
            assert window and all(re.search(r"\bsc1\b", l) for l in window), window
        wbl2 = [i for i, l in enumerate(lines) if l.startswith("buffer_wbl2") and "sc1" in l]
        inv = [i for i, l in enumerate(lines) if l.startswith("buffer_inv") and "sc1" in l]
        assert len(wbl2) >= 2 and len(inv) >= 2
        # the count of a finished item: write-back, then the atomic add, then invalidate
        adds = [i for i, l in enumerate(lines) if l.startswith("global_atomic_add")]
        assert any(any(w < a and a - w < 8 for w in wbl2) and any(a < v < a + 8 for v in inv) for a in adds)
        # the ready flag: a write-back right before an sc1 store
        stores = [i for i, l in enumerate(lines) if l.startswith("global_store_dword") and "sc1" in l]
        assert any(any(0 < s - w < 8 for w in wbl2) for s in stores)
