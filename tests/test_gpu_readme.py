"""The Python example of the README runs as written on the GPU and gives
finite results of the documented shapes."""
import os
import textwrap

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _readme_example():
    text = open(os.path.join(ROOT, "README.md")).read()
    sec = text.split("## Python use", 1)[1]
    lines = []
    for ln in sec.splitlines()[1:]:
        if ln.startswith("    ") or (ln.strip() == "" and lines):
            lines.append(ln)
        elif lines:
            break
    return textwrap.dedent("\n".join(lines))


@pytest.mark.skipif(not os.path.exists(os.path.join(ROOT, "README.md")), reason="README.md not in this tree")
def test_readme_python_example_runs():
    import torch
    code = _readme_example()
    assert "Sim(insts)" in code and "srv.submit" in code
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    sim, insts = ns["sim"], ns["insts"]
    B, n, T = len(insts), insts[0].n, insts[0].T
    nsz = 6 * n
    assert ns["traj"].numel() == B * (T + 1) * nsz and torch.isfinite(ns["traj"]).all()
    assert torch.isfinite(ns["s0_bar"]).all() and torch.isfinite(ns["u_bar"]).all()
    assert ns["A"].numel() == B * T * nsz * nsz and torch.isfinite(ns["A"]).all()
    assert ns["u"].grad is not None and torch.isfinite(ns["u"].grad).all()
    res = ns["res"]
    assert res.status == 0
    assert res.A is not None and res.A.shape == (T, nsz, nsz) and np.isfinite(res.A).all()
    assert res.u.shape == (T, insts[0].n_u)
    ns["srv"].close()
