"""Every bench.py option that the profiles, the design notes and the README cite exists,
so that the commands they give can be run again."""
import glob
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cited_bench_options_exist():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    known = set(re.findall(r"--[a-z0-9][a-z0-9-]*", r.stdout))
    docs = glob.glob(os.path.join(ROOT, "profiles", "*.md")) + \
        [os.path.join(ROOT, "DESIGN.md"), os.path.join(ROOT, "README.md")]
    missing = []
    for path in docs:
        text = open(path).read().replace("\\\n", " ")
        for m in re.finditer(r"bench\.py((?:\s+--[a-z0-9-]+(?:\s+[0-9A-Za-z_.]+)?)+)", text):
            for opt in re.findall(r"--[a-z0-9][a-z0-9-]*", m.group(1)):
                if opt not in known:
                    missing.append((os.path.relpath(path, ROOT), opt))
    assert missing == []
