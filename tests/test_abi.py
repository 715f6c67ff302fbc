"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every entry point include/fv.h declares, and rejects bad arguments on the host
before anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2302_09005_amd import fv
from paper_2302_09005_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(fv_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert "fv_batch_update" in names and "fv_max_eigenvalue" in names
    lib = fv.library()
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_supported_instances():
    assert fv.abi_version() == 1
    for d, p in [(2, 16), (2, 17), (3, 8), (3, 4), (3, 16)]:
        assert fv.supported(d, p)
    for d, p in [(3, 5), (2, 3), (4, 8), (1, 8)]:
        assert not fv.supported(d, p)


def test_descriptor_record_matches_header():
    src = open(os.path.join(ROOT, "include", "fv.h")).read()
    body = re.search(r"typedef struct fv_patch \{(.*?)\} fv_patch;", src, re.S).group(1)
    fields = re.findall(r"^\s*(int64_t|int32_t|double)\s+(\w+)(\[\d\])?;", body, re.M)
    assert [f[1] for f in fields] == list(W.PATCH_DTYPE.names)


def _grid_desc(out_halo=True):
    g = W.PatchGrid(3, 8, (2, 2, 2), 1 / 16)
    return g, g.descriptors(dt=1e-3, out_halo=out_halo)


def test_check_patches_accepts_valid_and_names_bad_patch():
    g, desc = _grid_desc()
    L = g.buffer_len(True)
    fv.check_patches(desc, 3, 8, True, L, L)
    bad = desc.copy()
    bad["q_in"][3] = L  # past the end
    with pytest.raises(fv.FVError, match="patch 3"):
        fv.check_patches(bad, 3, 8, True, L, L)
    bad = desc.copy()
    bad["p"][5] = 4
    with pytest.raises(fv.FVError, match="patch 5"):
        fv.check_patches(bad, 3, 8, True, L, L)
    bad = desc.copy()
    bad["q_out"][2] = bad["q_out"][1] + 8
    with pytest.raises(fv.FVError, match="overlap"):
        fv.check_patches(bad, 3, 8, True, L, L + 8)
    bad = desc.copy()
    bad["dx"][0, 1] = 0.0
    with pytest.raises(fv.FVError, match="dx"):
        fv.check_patches(bad, 3, 8, True, L, L)
    bad = desc.copy()
    bad["dt"][0] = np.nan
    with pytest.raises(fv.FVError, match="dt"):
        fv.check_patches(bad, 3, 8, True, L, L)
    g2, desc2 = _grid_desc(out_halo=False)
    fv.check_patches(desc2, 3, 8, False, L, g2.buffer_len(False))
    with pytest.raises(fv.FVError):
        fv.check_patches(desc2, 3, 8, False, L, g2.buffer_len(False) - 1)
    # compact input blocks
    desc3 = g2.descriptors(out_halo=False, in_halo=False)
    Lc = g2.buffer_len(False)
    fv.check_patches(desc3, 3, 8, False, Lc, Lc, q_in_halo=False)
    with pytest.raises(fv.FVError, match="input block"):
        fv.check_patches(desc3, 3, 8, False, Lc, Lc, q_in_halo=True)


def _call_update(**kw):
    a = dict(patches=0x1000, n=4, q_in=0x10000, q_in_len=1000, q_out=0x100000, q_out_len=1000,
             q_out_halo=1, dim=3, p=8, halo=1, s=5, gamma=1.4, dt=None, max_eig=None, stream=None)
    a.update(kw)
    lib = fv.library()
    return lib.fv_batch_update(a["patches"], a["n"], a["q_in"], a["q_in_len"], a["q_out"],
                               a["q_out_len"], a["q_out_halo"], a["dim"], a["p"], a["halo"],
                               a["s"], a["gamma"], a["dt"], a["max_eig"], a["stream"])


@pytest.mark.parametrize("kw,code", [
    (dict(dim=4), fv.FV_EINVAL),
    (dict(s=4), fv.FV_EINVAL),
    (dict(halo=2), fv.FV_EINVAL),
    (dict(p=0), fv.FV_EINVAL),
    (dict(p=5), fv.FV_EUNSUPPORTED),
    (dict(n=-1), fv.FV_EINVAL),
    (dict(gamma=1.0), fv.FV_EINVAL),
    (dict(gamma=float("nan")), fv.FV_EINVAL),
    (dict(q_out_halo=2), fv.FV_EINVAL),
    (dict(patches=None), fv.FV_EINVAL),
    (dict(q_in=None), fv.FV_EINVAL),
    (dict(q_out=0x10000 + 8 * 500), fv.FV_EINVAL),  # q_out overlaps q_in
])
def test_batch_update_rejects_bad_arguments_on_host(kw, code):
    assert _call_update(**kw) == code
    assert fv.library().fv_last_error().decode() != ""


def test_zero_patches_is_a_no_op_on_host():
    assert _call_update(n=0, patches=None, q_in=None, q_out=None) == fv.FV_OK


def test_other_entry_points_reject_bad_arguments_on_host():
    lib = fv.library()
    assert lib.fv_max_eigenvalue(0x1000, 4, 0x2000, 100, 1, 7, 3, 8, 5, 1.4, 0x3000, None,
                                 None) == fv.FV_EINVAL  # bad offsets selector
    assert lib.fv_max_eigenvalue(0x1000, 4, 0x2000, 100, 1, 0, 3, 8, 5, 1.4, None, None,
                                 None) == fv.FV_EINVAL  # per_patch required
    assert lib.fv_cfl_timestep(0x1000, 0, 0x2000, 3, 0.4, None, None, None) == fv.FV_EINVAL
    assert lib.fv_cfl_timestep(0x1000, 4, 0x2000, 3, -1.0, None, None, None) == fv.FV_EINVAL
    assert lib.fv_fill_halo(0x1000, 4, None, 0x2000, 100, 0, 3, 8, 1, 5, None) == fv.FV_EINVAL
    assert lib.fv_fill_halo(0x1000, 4, 0x3000, 0x2000, 100, 0, 3, 3, 1, 5,
                            None) == fv.FV_EUNSUPPORTED


def test_step_workspace_size_and_rejection_on_host():
    lib = fv.library()
    # 96 words (three 256-byte lines) per group of 64 workgroups, plus the top
    assert fv.step_workspace_words(4096, 3, 8) == 96 * (1 + 64)
    assert fv.step_workspace_words(64, 2, 16) == 96 * 2   # one patch (4 row chunks) per workgroup
    assert fv.step_workspace_words(100, 2, 16) == 96 * 3  # 100 workgroups: two groups + top
    assert fv.step_workspace_words(100, 2, 17) == 96 * 3  # one patch (3 row chunks) each
    assert fv.step_workspace_words(100, 2, 8) == 96 * 2   # 8 patches per workgroup: 13
    assert fv.step_workspace_words(0, 3, 8) == 0 and fv.step_workspace_words(10, 3, 5) == 0
    args = [0x1000, 4096, 0x2000, 0x10000, 1000, 0x100000, 1000, 3, 8, 5, 1.4, 0.4, 0x3000, None,
            0x4000]
    # too small a workspace is refused before any launch
    assert lib.fv_step_gather(*args, None, 0x5000, 2079, None) == fv.FV_EINVAL
    assert "workspace" in lib.fv_last_error().decode()
    # dt_next may not alias dt
    bad = list(args)
    bad[14] = 0x3000
    assert lib.fv_step_gather(*bad, None, 0x5000, 4096, None) == fv.FV_EINVAL


def test_step_pipelined_workspace_size_and_rejection_on_host():
    lib = fv.library()
    # three sets of 16 slots of 96 words (three 256-byte lines), any batch size
    assert fv.pipelined_workspace_words(4096, 3, 8) == 3 * 16 * 96
    assert fv.pipelined_workspace_words(100, 2, 8) == 3 * 16 * 96
    assert fv.pipelined_workspace_words(262144, 3, 8) == 3 * 16 * 96
    assert fv.pipelined_workspace_words(0, 3, 8) == 0
    assert fv.pipelined_workspace_words(10, 3, 5) == 0
    head = [0x1000, 4096, 0x2000, 0x10000, 1000, 0x100000, 1000, 3, 8, 5, 1.4, 0.4]
    tail = [None, None, None, None, 0x5000]
    f = lib.fv_step_gather_pipelined
    assert f(*head, 0, *tail, 3 * 16 * 96 - 1, None) == fv.FV_EINVAL
    assert "workspace" in lib.fv_last_error().decode()
    for phase in (-1, 3):
        assert f(*head, phase, *tail, 3 * 16 * 96, None) == fv.FV_EINVAL
        assert "phase" in lib.fv_last_error().decode()
    bad = list(head)
    bad[11] = 0.0  # cfl
    assert f(*bad, 0, *tail, 3 * 16 * 96, None) == fv.FV_EINVAL
    assert lib.fv_step_gather_pipelined_f32(*head, 0, None, None, None, None, None,
                                            3 * 16 * 96, None) == fv.FV_EINVAL  # null workspace
    bad = list(head)
    bad[1] = 0
    assert f(*bad, 0, *tail, 3 * 16 * 96, None) == fv.FV_EINVAL


def test_step_noalloc_refuses_batches_beyond_its_scratch_on_host():
    lib = fv.library()
    # 3-D 8^3: one patch per workgroup, 96 words per 64 workgroups plus 96
    limit = (393216 // 96 - 1) * 64
    assert limit == 262080
    assert fv.step_workspace_words(limit, 3, 8) == 393216
    assert fv.step_workspace_words(limit + 1, 3, 8) > 393216
    args = [0x1000, limit + 1, 0x2000, 0x10000, 1000, 0x100000, 1000, 3, 8, 5, 1.4, 0.4, 0x3000,
            None, 0x4000, None, None]
    assert lib.fv_step_gather_noalloc(*args) == fv.FV_EINVAL
    assert "scratch" in lib.fv_last_error().decode()
    bad = list(args)
    bad[1] = 8
    bad[14] = None  # dt_next is required
    assert lib.fv_step_gather_noalloc(*bad) == fv.FV_EINVAL
    bad = list(args)
    bad[1] = 8
    bad[9] = 4  # s != d + 2
    assert lib.fv_step_gather_noalloc(*bad) == fv.FV_EINVAL


def test_plan_mixed_sorts_by_size_and_fills_units():
    batch, _ = W.uneven_batch(300, 2)
    desc = batch.descriptors()
    plan = fv.Plan(desc, device="cpu")
    # stable sort, 16^3 first
    for p, first, count in plan.classes():
        idx = plan.order[first:first + count]
        assert (batch.sizes[idx] == p).all() and (np.diff(idx) > 0).all()
    assert sorted(plan.order.tolist()) == list(range(batch.n))
    assert [c[0] for c in plan.classes()] == [16, 8, 4]
    per_unit = {16: 1, 8: 4, 4: 16}
    u = plan.units_host
    assert plan.n_units == len(u) == sum(-(-c[2] // per_unit[c[0]]) for c in plan.classes())
    covered = []
    for rec in u:
        assert 1 <= rec["count"] <= per_unit[rec["p"]]
        idx = plan.order[rec["first"]:rec["first"] + rec["count"]]
        assert (batch.sizes[idx] == rec["p"]).all()
        covered += idx.tolist()
    assert sorted(covered) == list(range(batch.n))
    # biggest units first
    assert (np.diff([{16: 0, 8: 1, 4: 2}[int(p)] for p in u["p"]]) >= 0).all()


def test_plan_mixed_rejects_bad_batches():
    batch, _ = W.uneven_batch(10, 1)
    desc = batch.descriptors()
    bad = desc.copy()
    bad["p"][3] = 5
    with pytest.raises(fv.FVError, match="patch 3"):
        fv.Plan(bad, device="cpu")
    with pytest.raises(fv.FVError):
        fv.Plan(desc, device="cpu", dim=2)
    empty = fv.Plan(desc[:0], device="cpu")
    assert empty.n_units == 0 and empty.classes() == []


def _plan_struct(classes, n_units):
    c = fv.MixedPlan()
    c.order, c.units, c.n_units = 0x7000, 0x8000, n_units
    for k, (p, first, count) in enumerate(classes):
        c.class_p[k], c.class_first[k], c.class_count[k] = p, first, count
    return c


def test_step_local_rejects_bad_arguments_on_host():
    lib = fv.library()
    good = _plan_struct([(16, 0, 2), (8, 2, 5), (4, 7, 17)], 2 + 2 + 2)

    def call(plan=good, n=24, dim=3, s=5, gamma=1.4, cfl=0.4, schedule=1, wg=0, q_out=0x100000):
        return lib.fv_step_local(0x1000, n, 0x2000, ctypes.byref(plan), 0x10000, 1000, q_out,
                                 1000, dim, s, gamma, cfl, None, schedule, wg, None)
    assert call(dim=2) == fv.FV_EUNSUPPORTED
    assert call(s=4) == fv.FV_EINVAL
    assert call(cfl=0.0) == fv.FV_EINVAL
    assert call(gamma=1.0) == fv.FV_EINVAL
    assert call(schedule=3) == fv.FV_EINVAL
    assert call(wg=-1) == fv.FV_EINVAL
    assert call(n=25) == fv.FV_EINVAL and "covers" in lib.fv_last_error().decode()
    assert call(plan=_plan_struct([(16, 0, 2), (8, 2, 5), (4, 7, 17)], 7)) == fv.FV_EINVAL
    assert "work units" in lib.fv_last_error().decode()
    assert call(plan=_plan_struct([(16, 0, 2), (8, 3, 5), (4, 7, 17)], 6)) == fv.FV_EINVAL
    assert call(plan=_plan_struct([(16, 0, 2), (5, 2, 5), (4, 7, 17)], 6)) == \
        fv.FV_EUNSUPPORTED
    assert call(q_out=0x10000 + 8) == fv.FV_EINVAL          # overlapping buffers
    assert call(n=0) == fv.FV_OK                            # empty batch: no launch
    assert lib.fv_local_timestep(0x1000, 4, None, 3, 0.4, None) == fv.FV_EINVAL
    assert lib.fv_local_timestep(0x1000, 4, 0x2000, 3, -0.4, None) == fv.FV_EINVAL
    assert lib.fv_local_timestep(0x1000, 0, None, 3, 0.4, None) == fv.FV_OK


def test_learned_entry_points_reject_bad_arguments_on_host():
    lib = fv.library()
    # r must divide p; bc in {0, 1}; null pointers
    assert lib.fv_learned_flux_accumulate(0x1000, 4, 4, 16, 3, 0, 1.4, 0.25, 0x2000, 0x3000,
                                          None) == fv.FV_EINVAL
    assert lib.fv_learned_flux_accumulate(0x1000, 4, 4, 16, 4, 2, 1.4, 0.25, 0x2000, 0x3000,
                                          None) == fv.FV_EINVAL
    assert lib.fv_learned_flux_accumulate(None, 4, 4, 16, 4, 0, 1.4, 0.25, 0x2000, 0x3000,
                                          None) == fv.FV_EINVAL
    assert lib.fv_learned_coarse_grain(0x1000, 6, 4, 16, 4, 0x2000, None) == fv.FV_EINVAL
    assert lib.fv_learned_coarse_grain(0x1000, 4, 4, 16, 4, 0x1000, None) == fv.FV_EINVAL
    assert lib.fv_mlp_fit_normalization(0x1000, 10, 16, 2, None, 0, 0x2000, 0x3000,
                                        None) == fv.FV_EINVAL
    assert lib.fv_mlp_train_step(0x1000, 0x2000, 0, 1e-3, 0x3000, 0x4000, 100, 0x5000, 64,
                                 0x6000, 10 ** 6, None, None) == fv.FV_EINVAL  # step 0
    assert lib.fv_mlp_train_step(0x1000, 0x2000, 1, 1e-3, 0x3000, 0x4000, 100, 0x5000, 64,
                                 0x6000, 10, None, None) == fv.FV_EINVAL      # workspace
    assert "workspace" in lib.fv_last_error().decode()
    assert lib.fv_mlp_forward(0x1000, 0x2000, 0, 0x3000, None) == fv.FV_OK
    assert lib.fv_batch_update_learned_2d(0x1000, 4, 0x2000, 0x3000, 100, 0x3000 + 8, 100, 1.4,
                                          None, 0x4000, 0.2, None, None) == fv.FV_EINVAL
    assert lib.fv_batch_update_learned_2d(0x1000, 4, 0x2000, 0x3000, 100, 0x8000, 100, 1.4,
                                          None, 0x4000, -1.0, None, None) == fv.FV_EINVAL
    assert fv.mlp_workspace_words(1024) == 1024 * 277


def test_mlp_sizes_match_header_and_layout():
    from oracle import learned as OL
    src = open(os.path.join(ROOT, "include", "fv.h")).read()
    blob = int(re.search(r"#define FV_MLP_BLOB_WORDS (\d+)", src).group(1))
    trained = int(re.search(r"#define FV_MLP_TRAINED_WORDS (\d+)", src).group(1))
    sizes = {name: int(np.prod(shape)) for name, shape in OL.BLOB_LAYOUT}
    assert blob == fv.MLP_BLOB_WORDS == OL.BLOB_SIZE
    assert trained == fv.MLP_TRAINED_WORDS == sum(sizes[k] for k in ("w1", "b1", "w2", "b2",
                                                                    "w3", "b3"))
    o = 0
    for name, _ in OL.BLOB_LAYOUT:
        assert fv.BLOB_OFFSETS[name] == o
        o += sizes[name]


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_one_hip_runtime_in_the_process():
    """libfv binds to the HIP runtime torch loaded (the wheel ships its own
    copy under the same soname): after fv.library() the process maps exactly
    one libamdhip64, so torch's device memory and streams are valid in every
    libfv call whatever was imported first."""
    fv.library()
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(paths) == 1, paths
