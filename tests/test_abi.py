"""The C ABI library loads, exports every entry point of include/vgicp.h and
rejects bad arguments on the host before touching a device (CPU only)."""

import ctypes
import subprocess

import pytest

vg = pytest.importorskip("paper_2109_07073_amd.vgicp", reason="libvgicp.so not built")


def test_every_header_symbol_is_exported():
    names = vg.header_symbols()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", vg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = vg.lib()
    for n in names:
        assert getattr(lib, n) is not None
    assert set(vg._PROTOS) == set(names)


def test_version_and_last_error_never_null():
    lib = vg.lib()
    assert lib.vgicp_version() >= 200
    assert lib.vgicp_last_error(None) is not None


@pytest.mark.parametrize("row,what", [
    ((-1, 0, 0, 1), "src"), ((2, 0, 0, 1), "src"),
    ((0, -1, 0, 1), "tgt"), ((0, 3, 0, 1), "tgt"),
    ((0, 0, -1, 1), "pose_i"), ((0, 0, 4, 1), "pose_i"),
    ((0, 0, 0, 4), "pose_j"), ((0, 0, 0, -7), "pose_j"),
])
def test_validate_factors_rejects_out_of_range(row, what):
    with pytest.raises(vg.VgicpError) as ex:
        vg.validate_factors(2, 3, 4, [(0, 0, 0, 1), row])
    assert ex.value.code == vg.EINVAL
    assert "factor 1" in str(ex.value) and what in str(ex.value)


def test_validate_factors_accepts_good_and_empty_lists():
    vg.validate_factors(2, 3, 4, [(1, 2, 3, 0), (0, 0, 0, 0)])
    vg.validate_factors(0, 0, 0, [])


def test_validate_factors_null_and_negative_counts():
    lib = vg.lib()
    assert lib.vgicp_validate_factors(1, 1, 1, None, 3) == vg.EINVAL
    assert lib.vgicp_validate_factors(-1, 1, 1, None, 0) == vg.EINVAL
    assert lib.vgicp_validate_factors(1, 1, 1, None, -2) == vg.EINVAL


def test_null_handles_are_rejected_without_a_device():
    lib = vg.lib()
    h = ctypes.c_void_p()
    assert lib.vgicp_ctx_create(0, None, None) == vg.EINVAL
    assert lib.vgicp_voxelize(None, None, 0.5, ctypes.byref(h)) == vg.EINVAL
    assert lib.vgicp_map_info(None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_map_export(None, None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_factorset_create(None, None, 0, None, 0, None, 0, 0, 0, ctypes.byref(h)) == vg.EINVAL
    assert lib.vgicp_factorset_info(None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_linearize_factors(None, None, None, None, None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_evaluate_errors(None, None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_overlap(None, None, None, None, None) == vg.EINVAL
    assert lib.vgicp_ctx_synchronize(None) == vg.EINVAL
    assert lib.vgicp_ctx_set_stream(None, None) == vg.EINVAL
    # freeing NULL handles is allowed
    assert lib.vgicp_map_free(None) == vg.OK
    assert lib.vgicp_factorset_destroy(None) == vg.OK
    assert lib.vgicp_ctx_destroy(None) == vg.OK
    assert b"NULL" in lib.vgicp_last_error(None)


def test_context_creation_without_gpu_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = vg.lib()
    h = ctypes.c_void_p()
    rc = lib.vgicp_ctx_create(0, None, ctypes.byref(h))
    assert rc in (vg.EHIP, vg.EINVAL) and not h.value


def test_library_shares_the_hip_runtime_of_torch():
    """libvgicp.so must bind to the HIP runtime PyTorch already loaded; two HIP
    runtimes in one process do not share devices or pointers."""
    import os
    with open(f"/proc/{os.getpid()}/maps") as fh:
        libs = {line.split()[-1] for line in fh if "libamdhip64" in line}
    assert len(libs) == 1, libs


def test_server_rejects_bad_config_and_null_handles():
    lib = vg.lib()
    h = ctypes.c_void_p()
    opts = vg.COpts(0, 0, 0, 0, 0.0, 0)
    bad = [
        vg.CServerConfig(0, 0, 1000, 16, 2, 0, 0, opts),      # max_batch_factors
        vg.CServerConfig(0, 16, 0, 16, 2, 0, 0, opts),        # max_batch_points
        vg.CServerConfig(0, 16, 1000, 16, 0, 0, 0, opts),     # inflight
        vg.CServerConfig(0, 16, 1000, 16, 9, 0, 0, opts),     # inflight
        vg.CServerConfig(-1, 16, 1000, 16, 2, 0, 0, opts),    # budget
        vg.CServerConfig(0, 16, 1000, 16, 2, 100, 0, opts),   # tile_points
        vg.CServerConfig(0, 16, 1000, 16, 2, 0, 0, vg.COpts(7, 0, 0, 0, 0.0, 0)),
    ]
    for cfg in bad:
        assert lib.vgicp_server_create(0, ctypes.byref(cfg), ctypes.byref(h)) == vg.EINVAL
    assert lib.vgicp_server_create(0, None, ctypes.byref(h)) == vg.EINVAL
    assert lib.vgicp_server_destroy(None) == vg.OK
    assert lib.vgicp_server_memory(None, None, None) == vg.EINVAL
    assert lib.vgicp_server_poll(None, 1, None) == vg.EINVAL
    assert lib.vgicp_server_wait(None, 1, None) == vg.EINVAL
    assert lib.vgicp_server_remove_frame(None, 0) == vg.EINVAL
    assert lib.vgicp_server_stats(None, None, None, None, None) == vg.EINVAL
    tickets = (ctypes.c_int64 * 1)()
    assert lib.vgicp_server_submit_many(None, None, 0, tickets) == vg.EINVAL
    assert lib.vgicp_server_submit(None, 0, None, 0, None, 0, None, None, None, None, None,
                                   tickets) == vg.EINVAL


def test_bad_output_tensors_raise_before_any_library_call():
    """Caller-supplied outputs of linearize / evaluate / overlap are checked
    (dtype, shape, contiguity, device) before anything reaches the library:
    with a context and factor set whose handles are NULL, reaching the
    library would raise VgicpError, so a ValueError proves nothing ran."""
    from types import SimpleNamespace

    import torch

    from paper_2109_07073_amd import vgicp as vg
    ctx = SimpleNamespace(handle=None, device=0)
    fs = SimpleNamespace(handle=None, n_factors=3, n_poses=2, total_points=10)
    poses = torch.zeros((2, 12), dtype=torch.float64)
    good = {"H": torch.zeros((3, 12, 12), dtype=torch.float64),
            "b": torch.zeros((3, 12), dtype=torch.float64),
            "e": torch.zeros(3, dtype=torch.float64),
            "inliers": torch.zeros(3, dtype=torch.int64)}
    cases = [
        (vg.linearize_factors, dict(good, H=torch.zeros((2, 12, 12), dtype=torch.float64)), "shape"),
        (vg.linearize_factors, dict(good, e=torch.zeros(3, dtype=torch.float32)), "float64"),
        (vg.linearize_factors, {"H": good["H"]}, "missing"),
        (vg.evaluate_errors, {"e": good["e"], "inliers": good["e"]}, "int64"),
        (vg.evaluate_errors, {"e": torch.zeros(4, dtype=torch.float64)[::1][:3].clone()[:2],
                              "inliers": good["inliers"]}, "shape"),
        (vg.evaluate_errors, {"e": torch.zeros((3, 2), dtype=torch.float64)[:, 0],
                              "inliers": good["inliers"]}, "contiguous"),
        (vg.overlap, {"hits": good["inliers"], "overlap": good["inliers"]}, "float64"),
        (vg.overlap, {"hits": good["inliers"][:2], "overlap": good["e"]}, "shape"),
        # right dtype and shape, but host memory
        (vg.overlap, {"hits": good["inliers"], "overlap": good["e"]}, "CUDA"),
        (vg.evaluate_errors, {"e": good["e"], "inliers": good["inliers"]}, "CUDA"),
    ]
    for fn, out, what in cases:
        with pytest.raises(ValueError, match=what):
            fn(ctx, fs, poses, out=out)
    # graph replay needs caller-owned outputs
    with pytest.raises(ValueError, match="use_graph"):
        vg.linearize_factors(ctx, fs, poses, use_graph=True)
    with pytest.raises(ValueError, match="use_graph"):
        vg.evaluate_errors(ctx, fs, poses, use_graph=True)


def test_keyframe_calls_reject_null_handles_without_a_device():
    lib = vg.lib()
    r = vg._rules()
    d = ctypes.c_int32()
    c = vg.CCloud(None, None, 0)
    assert lib.vgicp_connect(None, ctypes.byref(c), None, None, None, 0, 0.025, 0, None, None,
                             None, None) == vg.EINVAL
    assert lib.vgicp_submap_step(None, ctypes.byref(r), ctypes.byref(c), None, None, None, None,
                                 None, 0, ctypes.byref(d), None, None) == vg.EINVAL
    assert lib.vgicp_server_connect(None, 0, None, None, None, 0, 0.025, 0, None, None, None,
                                    None) == vg.EINVAL
    assert lib.vgicp_server_submap_step(None, ctypes.byref(r), 0, None, 0, None, 0, None, 0,
                                        ctypes.byref(d), None, None) == vg.EINVAL


def test_binding_constants_match_the_header():
    """Every constant the Python binding mirrors has the header's value."""
    import re
    with open(vg.HEADER) as fh:
        text = fh.read()
    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"^#define (VGICP_\w+) \(?(-?\d+)\)?", text, re.M)}
    for name, value in (("OK", vg.OK), ("EINVAL", vg.EINVAL), ("ENOMEM", vg.ENOMEM),
                        ("ERANGE", vg.ERANGE), ("ENONFINITE", vg.ENONFINITE),
                        ("EHIP", vg.EHIP), ("EFULL", vg.EFULL),
                        ("NOALLOC_MAX_TILES", vg.NOALLOC_MAX_TILES)):
        assert defs["VGICP_" + name] == value, name
    groups = {"ACC": vg.ACC, "RESID": vg.RESID, "FUSED": vg.FUSED, "FORM": vg.FORM,
              "SCHED": vg.SCHED, "LAYOUT": vg.LAYOUT, "KERNEL": vg.KERNELS, "REQ": vg.REQ,
              "GATE": vg.GATE}
    for prefix, table in groups.items():
        header = {k[len("VGICP_" + prefix) + 1:].lower(): v for k, v in defs.items()
                  if k.startswith("VGICP_" + prefix + "_") and k != "VGICP_KERNEL_KINDS"}
        assert header == table, (prefix, header, table)
    header = {v: k[len("VGICP_SUBMAP_"):].lower() for k, v in defs.items()
              if k.startswith("VGICP_SUBMAP_")}
    assert header == vg.SUBMAP


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every struct the Python binding mirrors has the C compiler's size and
    field offsets for the header's typedef (a swapped or missing field in either
    would shift every later argument)."""
    import shutil
    import os
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"vgicp_cloud": vg.CCloud, "vgicp_factor": vg.CFactor, "vgicp_opts": vg.COpts,
               "vgicp_submap_rules": vg.CSubmapRules, "vgicp_server_config": vg.CServerConfig,
               "vgicp_server_request": vg.CServerRequest}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vgicp.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(vg.HEADER),
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_server_request_arrays_are_lent_to_one_request_at_a_time():
    """A finished request's host arrays may be reused by the next request, but
    never by two requests in flight (the worker would write both into them)."""
    class Srv:
        _inflight = {}
    srv = Srv()
    a = vg.ServerRequest(srv, "evaluate", 3)
    a.ticket = 1                                    # finished: not in flight
    b = vg.ServerRequest(srv, "evaluate", 3, out=a)
    assert b.inliers is a.inliers and b.e is a.e
    b.ticket = 2
    srv._inflight[2] = b
    with pytest.raises(ValueError):
        vg.ServerRequest(srv, "evaluate", 3, out=a)  # b still holds the arrays
    with pytest.raises(ValueError):
        vg.ServerRequest(srv, "evaluate", 3, out=b)  # b itself is in flight
    with pytest.raises(ValueError):
        vg.ServerRequest(srv, "linearize", 3, out=a)
    del srv._inflight[2]
    c = vg.ServerRequest(srv, "evaluate", 3, out=a)
    with pytest.raises(ValueError):                  # queued in the same call
        vg.ServerRequest(srv, "evaluate", 3, out=b, pending=[c])
