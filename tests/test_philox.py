"""The counter-based generator used for training frames, pinned to its
published known-answer vectors (CPU)."""
import json
import os

import numpy as np

from tests.helpers import philox4x32_10, philox_frame


def test_philox_known_answers():
    data = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "philox_kat.json")))
    for v in data["vectors"]:
        c = [int(h, 16) for h in v["ctr"]]
        k = [int(h, 16) for h in v["key"]]
        out = philox4x32_10(*[np.array([x]) for x in c], k[0], k[1])
        assert [int(o[0]) for o in out] == [int(h, 16) for h in v["out"]]


def test_philox_frame_statistics():
    x, nrm = philox_frame(200001, 7, 3, 0.5)
    assert x.shape == (200001,) and nrm.shape == (200001,)
    assert abs(x.mean() - 0.5) < 0.01
    assert abs(nrm.mean()) < 0.01 and abs(nrm.std() - 1.0) < 0.01
