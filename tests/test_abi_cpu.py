"""The C-ABI library on the host: it loads, exports every declared entry point, and rejects
inadmissible instances (appendix C, Part I(b): every commodity has a path and positive demand,
every used link positive capacity) without touching a GPU."""
import os
import re

import numpy as np
import pytest

import paper_2605_01748_amd as te
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = te.library()
    with open(os.path.join(ROOT, "include", "te.h")) as f:
        hdr = f.read()
    names = set(re.findall(r"\b(te_[a-z_]+)\s*\(", hdr))
    assert {"te_create", "te_solve", "te_grad", "te_solve_batch", "te_validate"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(te.API) == names


def test_default_options_match_header_defaults():
    o, _ = te.Options().to_c()
    assert np.isinf(o.alpha_target) and o.gamma == 1e-3 and o.beta0 == 1.0
    assert o.A == 10.0 and o.C == 2.0 and o.beta_every == 1 and o.project == 1 and o.ckpt_every == 16


def _inst():
    return W.make_instance("v", 3, [0, 1, 0], [1, 2, 2], [1.0, 2.0, 3.0], [0, 0], [2, 1], [1.0, 0.5],
                           [[[0, 1], [2]], [[0]]])


def test_valid_instance_passes():
    te.validate(_inst())
    te.validate(W.waxman20(0))


@pytest.mark.parametrize("mutate,needle", [
    (lambda i: setattr(i, "path_ptr", np.array([0, 2, 2, 3])), "empty"),
    (lambda i: i.path_links.__setitem__(0, 7), "out of range"),
    (lambda i: i.path_links.__setitem__(1, 0), "twice"),
    (lambda i: i.demand.__setitem__(1, 0.0), "must be finite and > 0"),
    (lambda i: i.demand.__setitem__(0, np.nan), "must be finite"),
    (lambda i: i.capacity.__setitem__(2, 0.0), "capacity"),
    (lambda i: i.capacity.__setitem__(1, np.inf), "not finite"),
    (lambda i: setattr(i, "demand_path_ptr", np.array([0, 2, 2], np.int32)), "expected n_paths"),
    (lambda i: setattr(i, "demand_path_ptr", np.array([0, 0, 3], np.int32)), "no path"),
    (lambda i: setattr(i, "path_ptr", np.array([1, 2, 3, 4])), "path_ptr[0]"),
])
def test_invalid_instances_rejected(mutate, needle):
    inst = _inst()
    mutate(inst)
    with pytest.raises(te.TEError) as ex:
        te.validate(inst)
    assert ex.value.status == te.TE_ERR_INVALID
    assert needle in str(ex.value)


def test_unused_link_may_have_zero_capacity():
    inst = W.make_instance("v", 3, [0, 1, 0], [1, 2, 2], [1.0, 2.0, 0.0], [0], [2], [1.0], [[[0, 1]]])
    te.validate(inst)


def test_too_many_paths_rejected():
    n = 65
    inst = W.make_instance("wide", 2, [0] * n, [1] * n, [1.0] * n, [0], [1], [1.0], [[[i] for i in range(n)]])
    with pytest.raises(te.TEError, match="at most 64"):
        te.validate(inst)


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(te.TEError) as ex:
        te.Problem(_inst())
    assert ex.value.status == te.TE_ERR_DEVICE


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of te_options and te_stats have the header's field offsets and sizes
    (checked by compiling the header with the host compiler)."""
    import ctypes
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = {"te_options": te._Options, "te_stats": te._Stats}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "te.h"', "int main(void) {"]
    for name, cls in fields.items():
        src.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            src.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(c), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    for name, cls in fields.items():
        assert int(out[f"{name} size"]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_dao_optimality_metric():
    """Section 4.1's optimality: mean over demands of min(X_d / max(OPT_d, theta), 1) -- rates above
    the optimum are not rewarded, theta guards zero optima."""
    from paper_2605_01748_amd import dao
    assert dao.optimality([1.0, 2.0], [1.0, 2.0], 1e-9) == 1.0
    assert dao.optimality([0.5, 4.0], [1.0, 2.0], 1e-9) == 0.75
    assert dao.optimality([0.0, 0.0], [1.0, 0.0], 1e-9) == 0.0
    assert dao.optimality([1e-10], [0.0], 1e-9) == pytest.approx(0.1)
    with pytest.raises(ValueError):
        dao.optimality([1.0], [1.0, 2.0], 1e-9)
