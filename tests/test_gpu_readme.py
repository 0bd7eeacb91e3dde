"""The Python example of README.md runs as written (keeps the documented API
in step with the binding)."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert blocks, "README.md has no Python example"
    for code in blocks:
        exec(compile(code, "README.md", "exec"), {})
