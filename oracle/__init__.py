"""Plain FP64 CPU oracle of the batched stellar-population forward model and logL.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls it, shares no code, tables or constants with it, and fails loudly
when its own compiled extension is missing.

Each function follows a passage of the paper (Stoffers et al., "Ceridwen: Fast
and Flexible GPU-Accelerated Stellar Population Inference"): the defining
formula is written out in float64 NumPy, in the paper's order and notation, with
no blocking, fusion or reordering beyond what the definition states.  Where the
paper leaves a detail open, the reading taken is stated in the docstring.

Modules:
  constants   physical constants (Sec. 2.6, App. E, App. F)
  cosmology   flat LambdaCDM distances and ages (Sec. 2.6)
  sfh         SFH/ZH -> SSP weights, step scheme (Sec. 2.2, App. B)
  nebular     ionising photon rate, line luminosities and grid profiles (Sec. 2.3, App. C)
  dust        two-component attenuation (Sec. 2.4, App. D.1)
  projection  photometry (App. E) and spectra (App. F)
  likelihood  diagonal Gaussian with noise floor (Sec. 4.1, App. G, App. H.2)
  model       the whole forward model for a batch of parameter vectors
  adjoint     hand-written reverse pass of ``model`` in FP64
"""
