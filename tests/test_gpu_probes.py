"""Roofline probes: every kind returns a positive figure; an unknown kind is
refused."""
import ctypes

import pytest

from paper_2508_16522_amd import taskgraph as tg

pytestmark = pytest.mark.gpu


def test_probes_positive(gpu):
    for kind in (tg.TG_PROBE_COPY_BW, tg.TG_PROBE_ATOMIC_DISTINCT, tg.TG_PROBE_ATOMIC_CONTENDED,
                 tg.TG_PROBE_LAUNCH_RATE, tg.TG_PROBE_HANDOFF_NS, tg.TG_PROBE_HANDOFF_SAME_XCD_NS,
                 tg.TG_PROBE_HANDOFF_FAR_XCD_NS, tg.TG_PROBE_HANDOFF_L2_NS):
        assert tg.tg_probe(kind) > 0, kind


def test_unknown_probe_refused(gpu):
    v = ctypes.c_double()
    assert tg.load().tg_probe(99, ctypes.byref(v)) == tg.TG_EINVAL
