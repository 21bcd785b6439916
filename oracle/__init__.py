"""FP64 CPU oracle for the QUEST FX-correlator hot path (arXiv 2604.20640).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; the two meet only at seeded inputs.

Each module states the passage of the paper it follows:

* :mod:`oracle.pfb`    -- F-engine: polyphase FIR + DFT (Sec. 4.1 step 1,
  Sec. 4.2 "F-engine", Alg. 1 "Apply PFB weighting -> FFT").
* :mod:`oracle.xengine` -- X-engine and integration (Sec. 4.1 eq. 1,
  Sec. 4.2 "X-engine and integration").
* :mod:`oracle.mad`    -- MAD flagging (Sec. 7, eq. 2).
* :mod:`oracle.calib`  -- delay/phase application (Sec. 4.1 step 2, eq. 1)
  and the three-step delay/phase solve (Sec. 7, steps 1-3, eq. 3).
* :mod:`oracle.quant`  -- reduced-precision quantisers used to build the
  quantisation-aware reference for the MFMA X-engine.
* :mod:`oracle.cnn`    -- the learned RFI flagger beside MAD (Sec. 5 RFI
  structure, Sec. 7 MAD): forward, backpropagation, loss, Adam.
* :mod:`oracle.imaging` -- synthesis imaging of Sec. 8.1: gridding, dirty
  image and beam, Hogbom CLEAN.

Everything is float64 (complex128) unless a function says otherwise.  Where
the paper is silent the reading taken is stated in the function docstring.
"""

from . import pfb, xengine, mad, calib, quant, cnn, imaging  # noqa: F401

__all__ = ["pfb", "xengine", "mad", "calib", "quant", "cnn", "imaging"]
