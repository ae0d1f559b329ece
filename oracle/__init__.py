"""CPU oracle of the mixture-of-experts layer -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy/SciPy code that the HIP library is
checked against.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does, and it imports nothing from the product package.

The paper this project accompanies defines no mixture-of-experts layer, so
no passage of it can be cited for these functions.  Every definition here is
a stated reading, written out in each module's header:

* ``routing``  -- FP32-replica router: capacity prices as LP dual variables,
  the ascending clearing-price update, price-adjusted top-k, gate weights,
  capacity enforcement; FP64 primal/dual objectives.
* ``certify``  -- brute-force enumeration, HiGHS LP and max-flow checks.
* ``ffn``      -- FP64 dispatch, SwiGLU experts and weighted combine.
* ``grad``     -- FP64 backward of the layer with the routing held fixed.
* ``fp8``      -- OCP e4m3 emulator and per-128-block quantisation.
* ``mlp``      -- FP64 price MLP (8-256-256-1, GELU) with Adam, and the
  eight per-expert logit statistics it reads.
"""
