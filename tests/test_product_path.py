"""The product path stands on the HIP library alone (CPU checks): the package
never imports the oracle, a missing library raises instead of falling back,
and bench.py refuses more than one GPU before touching one."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(code):
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                          timeout=120)


def test_package_does_not_import_the_oracle():
    r = _run("import sys, paper_2502_16818_amd, paper_2502_16818_amd.rollout\n"
             "print(sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')))")
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "[]"


def test_missing_library_raises():
    r = _run("import paper_2502_16818_amd.cdbm as c\n"
             "c.LIB_PATH = '/nonexistent/libcdbm.so'\n"
             "try:\n"
             "    c.load()\n"
             "except ImportError as e:\n"
             "    print('raised', e)\n")
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("raised")


def test_product_sources_name_no_oracle():
    """No HIP, C++ or Python source of the library refers to the oracle."""
    pkg = os.path.join(ROOT, "paper_2502_16818_amd")
    for d, _, files in os.walk(pkg):
        for name in files:
            if name.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(d, name)).read()
                assert "import oracle" not in text and "from oracle" not in text, name


@pytest.mark.parametrize("n", ["2", "8"])
def test_bench_refuses_several_gpus(n):
    r = subprocess.run([sys.executable, "bench.py", "--gpus", n], cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
