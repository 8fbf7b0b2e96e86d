"""The C-ABI library loads and exports every entry point of include/hww.h;
host-side validation (no GPU work) rejects bad problems."""
import os
import re

import numpy as np
import pytest

from paper_2512_19925_amd import hww as H
from paper_2512_19925_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hww.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hww_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 10
    L = H.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(H.EXPORTS) == names


def test_workspace_bytes_and_validation():
    w = W.plain_small()
    n = H.workspace_bytes(H.spec_from_workload(w))
    assert n > 0 and n % 256 == 0
    big = H.workspace_bytes(H.spec_from_workload(W.full_scale()))
    assert big > 8e9  # two 1.5x-padded banks of 4e7 particles plus queues
    bad = [
        dict(sigma_s=w.sigma_t * 1.5),                 # sigma_s > sigma_t
        dict(edges=w.edges[::-1].copy()),              # non-ascending
        dict(n_batches=0), dict(n_chunks=9), dict(dt=0.0), dict(speed=-1.0),
        dict(src_x=100.0), dict(bank_capacity=10), dict(precision=7),
    ]
    for kw in bad:
        spec = H.spec_from_workload(w)
        for k, v in kw.items():
            setattr(spec, k, v)
        with pytest.raises(H.HwwError) as ei:
            H.workspace_bytes(spec)
        assert ei.value.code == -1


def test_largest_mesh_is_accepted_and_one_more_cell_is_not():
    # The sweep keeps each work-group's tallies in LDS ([I][6] doubles):
    # 3136 cells fit with 2..8 chunks, 3137 do not.
    for I, ok in ((3136, True), (3137, False)):
        w = W.homogeneous(f"mesh-{I}", -1.0, 1.0, I, 1.0, 0.5, n_src=1000)
        if ok:
            assert H.workspace_bytes(H.spec_from_workload(w)) > 0
        else:
            with pytest.raises(H.HwwError) as ei:
                H.workspace_bytes(H.spec_from_workload(w))
            assert ei.value.code == -1


def _batch_bytes(specs):
    probs = (H.Problem * len(specs))(*[s.to_c() for s in specs])
    return H.lib().hww_batch_workspace_bytes(probs, len(specs))


def test_batch_workspace_bytes_and_validation():
    ws = W.batched_replicas(n_replicas=16)
    specs = [H.spec_from_workload(w) for w in ws]
    n = _batch_bytes(specs)
    assert n > 0 and n % 256 == 0
    # The batch holds every replica's banks and tallies.
    assert n > sum(w.n_src for w in ws) * 44 * 2
    # Replicas must share precision, chunk count and step count.
    for kw in (dict(n_chunks=3), dict(precision=H.HWW_FP32), dict(n_steps=7)):
        bad = list(specs)
        bad[5] = H.spec_from_workload(ws[5])
        for k, v in kw.items():
            setattr(bad[5], k, v)
        assert _batch_bytes(bad) == -1
    # An invalid replica invalidates the batch.
    bad = list(specs)
    bad[3] = H.spec_from_workload(ws[3])
    bad[3].n_batches = 0
    assert _batch_bytes(bad) == -1
    assert _batch_bytes([]) == -1


def test_fission_comb_and_tally_options_validation():
    w = W.paper_fission(n_src=2000)
    base = H.workspace_bytes(H.spec_from_workload(w))
    plain = H.workspace_bytes(H.spec_from_workload(w.with_(comb=0)))
    assert base > plain      # the comb's scratch and the wider daughter buffers
    bad = [
        dict(sigma_f=w.sigma_t * 0.9),                 # sigma_s + sigma_f > sigma_t
        dict(sigma_f=-w.sigma_f),                      # negative fission cross section
        dict(nu_f=-1.0), dict(nu_f=float("nan")),
        dict(comb=3), dict(comb=-1), dict(track_moments=4), dict(track_moments=-1),
    ]
    for kw in bad:
        spec = H.spec_from_workload(w)
        for k, v in kw.items():
            setattr(spec, k, v)
        with pytest.raises(H.HwwError) as ei:
            H.workspace_bytes(spec)
        assert ei.value.code == -1
    # Batches take neither fission nor combing.
    ws = W.batched_replicas(n_replicas=4)
    specs = [H.spec_from_workload(x) for x in ws]
    specs[2] = H.spec_from_workload(ws[2].with_(sigma_f=ws[2].sigma_t * 0.01, nu_f=2.0))
    assert _batch_bytes(specs) == -1
    specs[2] = H.spec_from_workload(ws[2].with_(comb=100))
    assert _batch_bytes(specs) == -1


def test_static_workspace_rejects_a_problem_too_big_for_it():
    # The size check comes before any device call, so it runs without a GPU.
    import ctypes as C
    L = H.lib()
    limit = 160 << 20
    for n_src, ok in ((10_000, True), (1_000_000, False)):
        spec = H.spec_from_workload(W.plain_small().with_(n_src=n_src))
        assert (H.workspace_bytes(spec) <= limit) == ok
    spec = H.spec_from_workload(W.plain_small().with_(n_src=1_000_000))
    p = spec.to_c()  # spec keeps the arrays p points into
    h = C.c_void_p()
    rc = L.hww_init_problem_static(C.byref(p), None, C.byref(h))
    assert rc == -1 and not h.value
    assert b"static workspace holds" in L.hww_last_error(None)
