"""Measurement support on the GPU: the generator-throughput entry point that
the sampler's ALU roofline is reported against."""
import pytest

from paper_2510_27117_amd import gfors


@pytest.mark.gpu
def test_generator_throughput_positive_and_arguments_checked():
    rate = gfors.philox_throughput(calls=1 << 26)
    assert rate > 1e9                      # well below any plausible device rate
    with pytest.raises(gfors.GforsError):
        gfors.philox_throughput(calls=0)
