"""CPU oracle for the batched tensor-network Monte Carlo hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything from here; the product path (the HIP
library and its Python binding) never does, and the oracle shares no code
with it.  Everything is float64 NumPy/LAPACK, slow and plain:

* philox.py  -- Philox4x32-10 (SC'11) and the 53-bit uniform conversion;
* ising.py   -- energy (Eq. 1), Boltzmann matrix (Eq. 7), spin packing;
* bmps.py    -- boundary-MPS cache build (section 3.2, dense MPO x MPS,
                QR then truncating SVD sweep);
* sampler.py -- row sampler with teacher forcing (section 3.3, Eqs. 3-5);
* mis.py     -- Metropolis independence chain (Eq. 10);
* exact.py   -- brute force and dense transfer vectors (the pins);
* mlp.py     -- float64 MLP forward/backward/Adam for the learned proposal
                correction (not part of the paper).

Parity status of each function and its pins is listed in each module header.
"""
