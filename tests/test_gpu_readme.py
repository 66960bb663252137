"""The README's Python examples run as written on the GPU."""
import os
import re

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_examples_run():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) >= 2
    scope = {}
    for code in blocks:
        exec(compile(code, "README.md", "exec"), scope)
    torch.cuda.synchronize()
    assert len(scope["norms"]) == 5 and scope["norms"][-1] < scope["norms"][0]
    assert scope["tiles"].shape[1] == 7
