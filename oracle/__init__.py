"""Plain, slow FP64 CPU reference of the relative-binned BNS likelihood.

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the GPU library is
checked against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the library and its Python binding never do.
It shares no code with the GPU path (the two share only the seeded input
generators in `synth`, which hold none of the method's arithmetic).

Every function follows the paper's definitions as directly as possible:
  * the Whittle likelihood and noise-weighted inner product (Sec. II A,
    Eqs. 2-3), discretised as a Riemann sum over the frequency grid;
  * relative binning (Sec. II C, Eqs. 4-5) taken step by step: reference
    waveform, per-bin summary data, ratio at the bin edges, linear model
    about the bin centre, sum over bins;
  * the TaylorF2 and IMRPhenomD_NRTidalv2 waveforms the paper analyses
    (Sec. II B), from the published post-Newtonian / phenomenological
    formulas;
  * gradients by forward-mode dual numbers through the same code.
"""
