"""FP64 CPU oracle of the matched-filter / projected-gradient hot path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct implementations
written from the paper's definitions (Section "Model-based MRF
reconstruction" eq. exactP and eq. blip, Algorithm 2, eq. steprule, the
DCF-weighted gradient eq. blip_dcf, Algorithm 1 for the cover tree).  Only
the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the GPU library never does, and the two share no code.
"""
