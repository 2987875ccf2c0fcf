import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def rocrand_philox():
    """Callable (seed, j, g) arrays -> rocRAND Philox4x32-10 words (host build)."""
    src = os.path.join(ROOT, "tests", "golden", "rocrand_philox_words.cpp")
    d = tempfile.mkdtemp(prefix="rocrand_philox_")
    exe = os.path.join(d, "rp")
    try:
        subprocess.run(["hipcc", "-O1", "-o", exe, src], check=True, cwd=d,
                       capture_output=True)
    except (OSError, subprocess.CalledProcessError) as e:  # pragma: no cover
        pytest.skip(f"cannot build rocRAND helper: {e}")

    def words(seeds, js, gs):
        lines = "".join(f"{int(s)} {int(j)} {int(g)}\n" for s, j, g in zip(seeds, js, gs))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True,
                             check=True).stdout.split()
        return [int(x) for x in out]

    return words
