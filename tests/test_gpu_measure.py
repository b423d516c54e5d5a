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


@pytest.mark.gpu
def test_streaming_read_reference_plausible_and_arguments_checked():
    """A bare 16-byte streaming read: positive and below the published 8 TB/s
    HBM peak (64 MiB, 1,024 workgroups); bad sizes are refused."""
    rate = gfors.read_throughput(nbytes=64 << 20, workgroups=1024)
    assert 1e11 < rate < 8.5e12
    with pytest.raises(gfors.GforsError):
        gfors.read_throughput(nbytes=64 << 20, workgroups=0)
