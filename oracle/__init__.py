"""FP64 CPU oracle of the Priori L+S iteration -- test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library.  Its functions are
pinned against closed forms, invariants and brute force in tests/test_oracle_pins.py.
Trajectories of noisy, undersampled problems beyond those pins are "parity
unpinned": the paper prints no values for them.
"""
from .priori_ls import (E, EH, fft3, ifft3, soft, haar_fwd, haar_inv, cas, uncas,  # noqa: F401
                        sv_targets, svt, svt_gram, sparse_step, dc_step, solve, plain_ls,
                        psnr, rel_l2, NULL_REL, shift_window, append_frame,
                        tfft_fwd, tfft_inv, db4_fwd, db4_inv, DB4_H, DB4_G, T_fwd, T_inv,
                        TRANSFORMS, set_fft_workers)
