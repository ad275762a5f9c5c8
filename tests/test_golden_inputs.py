"""The synthetic inputs against the ranges the paper prints (no GPU): the prior boxes of
Tab. II and the waveform-accuracy ranges of Tab. I, read from tests/golden, bound every
parameter the seeded generators draw, and the boxes are the printed ones."""
import os

import numpy as np

import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


SYMBOLS = {"pi": np.pi, "2pi": 2 * np.pi}


def _read(name):
    rows = {}
    for line in open(os.path.join(HERE, name)):
        line = line.split("#")[0].split()
        if line:
            rows[line[0]] = [SYMBOLS[t] if t in SYMBOLS else float(t) for t in line[1:]]
    return rows


def test_prior_boxes_are_the_printed_ones():
    t = _read("tab2_priors.txt")
    keys = {"Mc": "Mc", "q": "q", "chi": "chi", "Lambda": "L", "dL": "dL", "tc": "tc"}
    for col, prior in enumerate(("injection", "gw170817", "gw190425")):
        for name, key in keys.items():
            assert synth.PRIORS[prior][key] == (t[name][2 * col], t[name][2 * col + 1]), (prior, name)


def test_prior_draws_stay_in_the_printed_boxes():
    t = _read("tab2_priors.txt")
    for col, prior in enumerate(("injection", "gw170817", "gw190425")):
        th = synth.draw_theta(5 + col, 20000, prior)
        lo = lambda n: t[n][2 * col]  # noqa: E731
        hi = lambda n: t[n][2 * col + 1]  # noqa: E731
        checks = [("Mc", th[:, 0]), ("q", th[:, 1]), ("chi", th[:, 2]), ("chi", th[:, 3]), ("Lambda", th[:, 4]),
                  ("Lambda", th[:, 5]), ("dL", th[:, 6]), ("tc", th[:, 7]), ("phic", th[:, 8]),
                  ("cosi", np.cos(th[:, 9])), ("psi", th[:, 10]), ("ra", th[:, 11]), ("sindec", np.sin(th[:, 12]))]
        for name, v in checks:
            assert v.min() >= lo(name) - 1e-12 and v.max() <= hi(name) + 1e-12, (prior, name)
            # uniform over the box: the draws reach both ends (within 1 % of its width)
            w = hi(name) - lo(name)
            assert v.min() < lo(name) + 0.01 * w and v.max() > hi(name) - 0.01 * w, (prior, name)


def test_mismatch_draws_stay_in_the_printed_ranges():
    t = _read("tab1_mismatch_ranges.txt")
    th = synth.mismatch_draws(3, 20000)
    mc, q = th[:, 0], th[:, 1]
    # back to component masses: q = m2 / m1, Mc = (m1 m2)^(3/5) / (m1 + m2)^(1/5)
    m1 = mc * (1 + q) ** 0.2 / q ** 0.6
    m2 = q * m1
    for name, v in (("m", m1), ("m", m2), ("chi", th[:, 2]), ("chi", th[:, 3]), ("Lambda", th[:, 4]),
                    ("Lambda", th[:, 5]), ("iota", th[:, 9])):
        lo, hi = t[name]
        assert v.min() >= lo - 1e-9 and v.max() <= hi + 1e-9, name
        assert v.min() < lo + 0.01 * (hi - lo) and v.max() > hi - 0.01 * (hi - lo), name
