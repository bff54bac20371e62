"""TEST INFRASTRUCTURE: the CPU oracle.

A plain, slow, independent reference for what the GPU path computes.  Only
tests/, the package smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does.

  ckks_oracle.c  RNS-CKKS integer arithmetic (C, __int128 %, textbook NTT)
  ckks.py        ctypes front end, level/scale bookkeeping
  encode.py      FP64 canonical-embedding encode/decode (numpy FFT)
  circuit.py     one encrypted QG-NAG iteration, op by op
  trainer.py     FP64 plaintext QG-NAG (the method's definition)
  sigfit.py      FP64 least-squares / gradient reference for the learned sigmoid
"""
