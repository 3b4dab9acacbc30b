"""Host-side parts of the request loop (no GPU): the seeded arrival process."""
import numpy as np


def test_arrivals_follow_the_rate():
    from paper_1209_0410_amd.serve import sinusoidal_arrivals
    t = sinusoidal_arrivals(60.0, 1000, 20000, 60.0, seed=7)
    assert (np.diff(t) >= 0).all() and t.min() >= 0 and t.max() <= 60
    # expected count = mean rate x duration = 10,500 x 60
    assert abs(len(t) - 630_000) < 5 * np.sqrt(630_000)
    # the rate is lowest at the ends of the period and highest in the middle
    c = np.histogram(t, bins=6, range=(0, 60))[0]
    assert c[2] > 3 * c[0] and c[3] > 3 * c[5]
