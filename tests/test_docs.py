"""Every file that README.md or the design doc names in backquotes exists (paths relative to
the repository, the package, its csrc/ or tests/; brace lists and globs expanded; built
libraries are not checked)."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BASES = ("", "paper_1401_1112_amd", os.path.join("paper_1401_1112_amd", "csrc"), "tests")


def _expand(p):
    m = re.search(r"\{([^}]*)\}", p)
    if not m:
        return [p]
    return [q for alt in m.group(1).split(",") for q in _expand(p[:m.start()] + alt + p[m.end():])]


def _named_files(doc):
    text = open(os.path.join(ROOT, doc)).read()
    for tok in re.findall(r"`([^`\s]+)`", text):
        path = tok.split("::")[0]
        if re.search(r"\.(py|hip|h|cpp|json|txt|md)$|/$", path):
            yield from _expand(path)


@pytest.mark.parametrize("doc", ["README.md", "DESIGN.md"])
def test_named_files_exist(doc):
    missing = [p for p in _named_files(doc)
               if not any(glob.glob(os.path.join(ROOT, b, p)) for b in BASES)]
    assert not missing, missing
