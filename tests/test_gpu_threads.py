"""Host threads calling the library at once (marked `gpu`): total viewsheds of grids whose sweep rows
need different amounts of LDS, each thread on its own stream, give the same maps as one at a time."""
import sys
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tvs():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2003_02200_amd as t

    t.lib()
    return t


def test_threads_with_different_row_lengths(tvs):
    import torch

    # rows of 2000, 9000 and 15000 doubles: about 17, 74 and 123 KB of workgroup LDS
    shapes = [(40, 2000), (3, 9000), (2, 15000)]
    rng = np.random.default_rng(77)
    dems = [torch.from_numpy((500.0 + rng.normal(0.0, 3.0, s).cumsum(axis=1)).astype(np.float32)).cuda()
            for s in shapes]
    note("threads: serial reference")
    ref = [tvs.total_viewshed(d, 10.0, 1.5, 2, 1500.0).cpu() for d in dems]
    errors = []

    def work(x):
        try:
            st = torch.cuda.Stream()
            for _ in range(3):
                with torch.cuda.stream(st):
                    out = tvs.total_viewshed(dems[x], 10.0, 1.5, 2, 1500.0, stream=st)
                st.synchronize()
                if not torch.equal(out.cpu(), ref[x]):
                    errors.append(f"grid {shapes[x]} differs")
        except Exception as e:  # reported below, on the main thread
            errors.append(f"grid {shapes[x]}: {e}")

    note("threads: concurrent calls")
    ts = [threading.Thread(target=work, args=(x,)) for x in range(len(shapes))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
