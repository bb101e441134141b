"""CPU checks of the C-ABI library: it loads, exports every function that
include/tr.h declares, maps a single HIP runtime next to torch, computes the
mode schedule on the host exactly as the oracle does, and rejects bad
arguments in host validation.  No kernel is launched."""
import os
import re
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tr.h")
LIB = os.path.join(ROOT, "paper_2303_16492_amd", "libtrsgd.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\*?\s+\*?(tr_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("tr_sample", "tr_subchain", "tr_grad", "tr_update", "tr_relerr", "tr_run",
                 "tr_dist", "tr_dist_optimal", "tr_entry_fwd", "tr_entry_bwd"):
        assert must in names


def test_every_declared_symbol_is_exported():
    from paper_2303_16492_amd import _lib
    h = _lib.lib()
    missing = [n for n in _declared() if not hasattr(h, n)]
    assert not missing, missing


def test_single_hip_runtime_mapped():
    code = textwrap.dedent(f"""
        import sys; sys.path.insert(0, {ROOT!r})
        from paper_2303_16492_amd import _lib
        _lib.lib()
        maps = open('/proc/self/maps').read()
        paths = sorted({{l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}})
        print(len(paths), paths)
        assert len(paths) == 1, paths
    """)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr


def test_host_mode_pick_equals_oracle():
    from oracle import sampling
    from paper_2303_16492_amd import api
    for seed in (0, 1, 12345, 2**63 + 7):
        for N in (2, 3, 5, 8):
            for t in list(range(50)) + [10**6, 2**40 + 3]:
                assert api.tr_mode(seed, t, N) == sampling.pick_mode(seed, t, N)


def test_abi_version_and_status_strings():
    from paper_2303_16492_amd import _lib
    h = _lib.lib()
    assert h.tr_abi_version() == 2
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -99):
        assert len(h.tr_status_str(s)) > 0


def test_host_validation_rejects_bad_arguments():
    """Run in a child with no GPU visible: a validation bug could then never
    reach a kernel with the fake pointers used here."""
    code = textwrap.dedent(f"""
        import sys, ctypes as C; sys.path.insert(0, {ROOT!r})
        import torch
        from paper_2303_16492_amd import _lib as L, api
        h = L.lib()
        fake = C.c_void_p(4096)
        d = api.make_desc([4, 5, 6], [2, 3, 2], torch.float32)
        # order out of range
        bad = api.make_desc([4, 5, 6], [2, 3, 2], torch.float32); bad.N = 1
        assert h.tr_sample(C.byref(bad), 0, 0, 0, 4, None, None, 1, fake, fake, None) == -2
        bad.N = 9
        assert h.tr_subchain(C.byref(bad), 0, None, fake, 4, fake, None) == -2
        # rank above the maximum
        bad = api.make_desc([4, 5, 6], [2, 17, 2], torch.float32)
        assert h.tr_sample(C.byref(bad), 0, 0, 0, 4, None, None, 1, fake, fake, None) == -2
        # null descriptor / outputs / mode out of range
        assert h.tr_sample(None, 0, 0, 0, 4, None, None, 1, fake, fake, None) == -1
        assert h.tr_sample(C.byref(d), 0, 0, 0, 4, None, None, 1, None, fake, None) == -1
        assert h.tr_sample(C.byref(d), 0, 0, 3, 4, None, None, 1, fake, fake, None) == -1
        assert h.tr_sample(C.byref(d), 0, 0, -1, 4, None, None, 1, fake, fake, None) == -1
        # misaligned output
        assert h.tr_sample(C.byref(d), 0, 0, 0, 4, None, None, 1, C.c_void_p(4098), fake, None) == -4
        # dtype combination: FP64 cores with FP32 X
        bad = api.make_desc([4, 5, 6], [2, 3, 2], torch.float64, torch.float32)
        assert h.tr_subchain(C.byref(bad), 0, None, fake, 4, fake, None) == -3
        # precision not matching the cores
        cores = (C.c_void_p * 8)(4096, 4096, 4096)
        assert h.tr_grad(C.byref(d), 0, fake, fake, fake, fake, fake, 4, 0, fake, None, None,
                         fake, 1 << 30, None) == -3
        # workspace too small
        need = h.tr_grad_workspace_size(C.byref(d), 64, 1)
        assert need > 0
        assert h.tr_grad(C.byref(d), 0, fake, fake, fake, fake, fake, 64, 1, fake, None, None,
                         fake, need - 1, None) == -5
        # AdaGrad without its accumulator; bad rule kind; negative damping
        r = api.step_rule("adagrad")
        assert h.tr_update(C.byref(d), 0, fake, fake, None, 0.0, C.byref(r), 0, None, None,
                           fake, 1 << 20, None) == -1
        r = api.step_rule(); r.kind = 7
        assert h.tr_update(C.byref(d), 0, fake, fake, None, 0.0, C.byref(r), 0, None, None,
                           fake, 1 << 20, None) == -1
        r = api.step_rule()
        assert h.tr_update(C.byref(d), 0, fake, fake, None, -1.0, C.byref(r), 0, None, None,
                           fake, 1 << 20, None) == -1
        # laws: tr_dist refuses the uniform and optimal codes
        assert h.tr_dist(C.byref(d), 0, 0, fake, fake, None, fake, 1 << 20, None) == -1
        assert h.tr_dist(C.byref(d), 0, 3, fake, fake, None, fake, 1 << 20, None) == -1
        # run without a step counter
        p = L.tr_problem(); p.desc = d
        c = L.tr_config(); c.m = 8
        assert h.tr_run(C.byref(p), C.byref(c), None, 1, None, None, fake, 1 << 20, None) == -1
        # entry-point sizes stay defined for bad input
        assert h.tr_grad_workspace_size(None, 64, 1) == 0
        print("ok")
    """)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_batch_upload_rejects_bad_items_before_any_device_call():
    """Host validation of tr_batch_upload / tr_batch_run in a child with no
    GPU visible: every case fails before the copy or the launch."""
    code = textwrap.dedent(f"""
        import sys, ctypes as C; sys.path.insert(0, {ROOT!r})
        import torch
        from paper_2303_16492_amd import _lib as L, api
        h = L.lib()
        def item(I, R, xdt=torch.float16, reps=True, t=True, rule="fixed"):
            it = L.tr_batch_item()
            it.desc = api.make_desc(I, R, torch.float32, xdt)
            for k in range(len(I)):
                it.cores[k] = 4096 * (k + 1)
                it.Xrep[k] = 8192 * (k + 1) if reps else None
            it.t_dev = 256 if t else None
            it.m, it.rule, it.seed = 16, api.step_rule(rule, alpha=0.1), 1
            return it
        table = C.c_void_p(1 << 20)
        size = h.tr_batch_table_size(1)
        assert size >= C.sizeof(L.tr_batch_item)
        def up(it):
            return h.tr_batch_upload((L.tr_batch_item * 1)(it), 1, table, size, None)
        assert up(item([8, 9, 10], [2, 3, 2], xdt=torch.float32)) == -3   # X must be FP16
        assert up(item([8, 9, 200], [2, 3, 2])) == -2                      # I_n above 128
        assert up(item([8, 9, 10], [13, 3, 2])) == -2                      # R_n above 12
        assert up(item([8, 9, 10], [2, 3, 2], reps=False)) == -1           # replicas required
        assert up(item([8, 9, 10], [2, 3, 2], t=False)) == -1              # step counter required
        assert up(item([8, 9, 10], [2, 3, 2], rule="adagrad")) == -1       # accumulators required
        assert h.tr_batch_upload((L.tr_batch_item * 1)(item([8, 9, 10], [2, 3, 2])), 1, table, size - 1,
                                 None) == -5
        assert h.tr_batch_run(table, 1, 1, 48, 4, None) == -1              # chunk not offered
        assert h.tr_batch_run(table, 1, 1, 64, 6, None) == -1              # waves not offered
        assert h.tr_batch_run(C.c_void_p((1 << 20) + 8), 1, 1, 64, 4, None) == -4
        wsz = h.tr_batch_split_workspace_size(1, 4)
        assert wsz > 0 and h.tr_batch_split_workspace_size(1, 17) == 0
        ws = C.c_void_p(1 << 24)
        assert h.tr_batch_run_split(table, 1, 1, 64, 4, 0, ws, wsz, None) == -1       # splits 1..16
        assert h.tr_batch_run_split(table, 1, 1, 64, 4, 17, ws, wsz, None) == -1
        assert h.tr_batch_run_split(table, 1, 1, 48, 4, 4, ws, wsz, None) == -1       # chunk not offered
        assert h.tr_batch_run_split(table, 1, 1, 64, 4, 4, ws, wsz - 1, None) == -5   # workspace too small
        assert h.tr_batch_run_split(table, 1, 1, 64, 4, 4, C.c_void_p((1 << 24) + 8), wsz, None) == -4
        print("ok")
    """)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
