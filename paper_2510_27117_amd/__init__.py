"""GFORS hot path for MI355X (gfx950): PDHG + Philox Bernoulli sampling +
exact candidate evaluation, behind the C ABI of include/gfors.h.

Import the binding explicitly (``from paper_2510_27117_amd import gfors``);
importing the package itself loads nothing."""
