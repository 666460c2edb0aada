"""The render kernel's fast correctly rounded reciprocal and square root
(hardware approximation plus a fused-residual correction) against the
compiler's correctly rounded division and square root, on every binary32
input of their domains, on the device.  The kernel and the oracle trace the
same paths only if every division and square root on the geometric chain is
correctly rounded on both sides."""
import pytest

pytestmark = pytest.mark.gpu


def test_fast_reciprocal_and_sqrt_are_correctly_rounded_on_every_input():
    from paper_2211_17263_amd import native as NV
    print("[case] math self-test over 2^32 inputs", flush=True)
    ctx = NV.Context(0)
    try:
        bad = NV.prdpt_selftest_math(ctx)
    finally:
        ctx.close()
    assert bad == (0, 0, 0), dict(zip(("recip_nr", "sqrt_nr", "sqrt_cr"), bad))
