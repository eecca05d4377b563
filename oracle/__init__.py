"""CPU oracle for structure-aware irregular blocked sparse LU.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call or link anything in this
package.  The product library never routes through it.

It is a plain, slow, obviously correct implementation of what the solve path
computes, written from the paper and from textbook definitions:

* ``ordering``  -- fill-reducing permutation (the paper names none, Section 1
  and Section 2.1; a geometric nested dissection with a fixed rule is used);
* ``symbolic``  -- the filled, structurally symmetric pattern S of the factors
  (Section 1 phase 2, Section 4.2);
* ``blocking``  -- the diagonal block pointer (Algorithm 2), the nonzero
  percentage curve and its 1000-point sampling (Section 4.2/4.3), the
  irregular blocking (Algorithm 3) and regular blocking (Section 3.2);
* ``numeric``   -- the no-pivot right-looking LU of the permuted matrix on S
  (the scalar form of Algorithm 1), forward/backward solves and their
  transposes, in fp64, in plain C compiled with gcc;
* ``metrics``   -- flop count and normwise backward error.

It shares no code with the GPU path; the seeded matrix generators live in the
separate ``synth`` module, which holds none of the method's arithmetic.
"""
