"""Plain, slow CPU FP64 oracle of the long-characteristics transport sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the HIP library.

It computes, in the order and notation of the paper's section on the method
of long characteristics:

* ``rays``    -- the characteristic grid: per direction, parallel
                 characteristics of width w_k cut into segments at cell
                 boundaries (all grid-line crossings found and sorted, then
                 merged), in the uniform-spacing form and in the paper's
                 vertex-avoiding, width-halving form;
* ``sweep``   -- eq. (10)-(13): backward-Euler source Q, modified opacity,
                 segment propagation, optical thickness, the weight alpha and
                 segment-average intensities;
* ``moments`` -- eq. (7), (14)-(16): area-weighted cell averages, the angular
                 moments E, F and the Eddington tensor, plus boundary factors;
* ``solve``   -- the time loop with prescribed material data;
* ``faces``, ``closures`` -- face-average Eddington tensors (eq. (16)) and
                 the grey spectrum averages of eq. (8)-(9);
* ``loqd``    -- the multigroup and effective grey low-order equations,
                 eq. (4)-(6), in a finite-volume reading;
* ``material``, ``mlqd`` -- the Fleck-Cummings material and one time step
                 of the multilevel method (transport, multigroup and grey
                 levels, iterated).

Parity pins (tests/test_oracle_*.py) tie every function to what the paper and
the mathematics fix; the functions with no such pin say "parity unpinned" in
their docstrings.
"""
from . import rays, sweep, moments, solve  # noqa: F401
