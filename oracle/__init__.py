"""CPU oracle for DKSS multiplication (test infrastructure, not product code).

Plain, slow, obviously-correct implementations of what the GPU path computes,
written from the thesis (Lüders, "Fast Multiplication of Large Integers:
Implementation and Analysis of the DKSS Algorithm", Ch. 2-4).  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import, call, link or execute anything in this package.  It shares no code
with ``paper_1503_04955_amd`` and never imports it.

Modules
  params   parameter rule, Proth prime, generator, Hensel lift, omega, rho (Python ints)
  brute    tiny brute-force references (naive DFT over R, Kronecker-Schoenhage, Python-int products)
  coracle  ctypes binding of dkss_oracle.c: schoolbook, ring arithmetic, FFT over R,
           encode / pointwise / decode, residues, and the whole DKSS pipeline
  smul     Schoenhage-Strassen multiplication modulo 2^N + 1 (Sec. 2.9) in Python integers: the
           transform over Z/(2^K + 1)Z, the weighted (negacyclic) procedure and the outermost
           full-product form
"""
