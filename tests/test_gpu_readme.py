"""The Python example in README.md runs as written, and its results solve
what its comments say they solve."""

import os
import re

import numpy as np
import pytest
import torch

from oracle import wilson

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example():
    with open(os.path.join(ROOT, "README.md")) as f:
        code = re.search(r"```python\n(.*?)```", f.read(), re.S).group(1)
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    U = ns["U"].detach().cpu().numpy()
    psi = ns["psi"].cpu().numpy()
    m = ns["m"]
    chi = ns["chi"].cpu().numpy()
    ref = wilson.dslash(U, psi, m)
    assert np.max(np.abs(chi - ref)) <= 1e-13 * np.max(np.abs(ref))
    y = ns["y"].detach().cpu().numpy()
    r = np.linalg.norm((psi - wilson.dslash(U, y, m)).ravel()) / np.linalg.norm(psi.ravel())
    assert r < 1e-11
    assert all(s["status"] == 0 for s in ns["st"])
