"""The Python examples of README.md run as written on the GPU (the blocks
are executed in order in one namespace), so the documented calls stay
valid."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_examples_run():
    import torch
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) >= 2
    ns = {}
    for b in blocks:
        exec(compile(b, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    # the examples' results are what they say
    x, z = ns["x"], ns["z"]
    assert torch.allclose(z, x, atol=1e-5)
    assert ns["bins"].shape == (16, 2048, 1025)
    assert ns["ys"].numel() == sum(ns["sizes"])
    assert ns["res"]["code"].shape == (2, 128 * 128)
