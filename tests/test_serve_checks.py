"""Host-side checks of the counting server (no GPU): malformed jobs are
refused at submission, before they could share a batch with other jobs."""
import numpy as np
import pytest

from paper_1305_1861_amd.serve import Job, Server

GOOD = dict(bases=np.frombuffer(b"ACGTACGTAC", np.uint8).copy(), offsets=np.array([0, 4, 10], np.uint64), k=3, c=2)


def test_good_job_accepted():
    Server.check_job(Job(**GOOD))


@pytest.mark.parametrize("field,value", [
    ("offsets", np.array([0, 4, 12], np.uint64)),   # past its bases: would cut the next job's windows
    ("offsets", np.array([1, 4, 10], np.uint64)),
    ("offsets", np.array([0, 6, 4, 10], np.uint64)),
    ("offsets", np.array([0, 4, 10], np.int32)),
    ("offsets", np.zeros(0, np.uint64)),
    ("bases", np.zeros(10, np.int16)),
    ("k", 0), ("k", 64), ("c", 0), ("c", -1),
])
def test_malformed_job_refused(field, value):
    job = dict(GOOD)
    job[field] = value
    with pytest.raises(ValueError):
        Server.check_job(Job(**job))
