"""The Python example of README.md, run as written on the 256^3 workload's
fields (mixed precision: b in float32): it plans, reads dt_par, takes one
super-step of 16 stages and leaves a finite, changed temperature."""
import os
import re

import pytest

from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert len(blocks) == 1
    n = (256, 256, 256)
    T = inputs.noisy_temperature(n, 2, device="cuda:0")
    b = inputs.tangled_b(n, 1, device="cuda:0").float().contiguous()
    T0 = T.clone()
    scope = {"T": T, "b": b}
    print("running the README example", flush=True)
    exec(blocks[0], scope)
    assert scope["s"] == 16
    assert bool(torch.isfinite(T).all()) and not torch.equal(T, T0)
    scope["plan"].close()
