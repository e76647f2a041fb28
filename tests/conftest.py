import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")


def load_blocks(name):
    """Parse a golden fixture made of [name] blocks of whitespace rows."""
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            if ln.startswith("["):
                cur = ln[1:-1]
                blocks[cur] = []
                continue
            blocks[cur].append(ln.split())
    return blocks


def load_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                rows.append([int(x) for x in ln.split()])
    return rows


def lower_table(rows):
    """[(i, k) -> int] from a block of rows with '-' above the diagonal."""
    out = {}
    for i, r in enumerate(rows, 1):
        for k, v in enumerate(r, 1):
            if v != "-":
                out[(i, k)] = int(v)
    return out
