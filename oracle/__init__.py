"""FP64 CPU oracle for the WaveOrder hot path (arXiv 2412.09775).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_2412_09775_amd``) never imports, links or calls anything here, and this
package never imports the GPU library: the two share no code.

Everything is plain NumPy/SciPy in float64 / complex128, written to be read
against the paper:

* ``optics``   -- frequency grids, illumination pupil S, detection pupil P,
                  scalar Green's spectrum, propagators (Methods, "Summary of
                  transfer functions").
* ``tf``       -- transfer functions as autocorrelations of pupils (Table 1,
                  scalar column), the 5-channel polarisation bank, the thin
                  (phase-from-defocus) model.
* ``vector``   -- the vector label-free bank (Table 1, vector column): tensor
                  pupils, the Green's tensor spectrum, spherical-harmonic
                  object tensors and Stokes / analyser channels.
* ``linear``   -- forward model D = sum_p H_cp F_p + b delta (Methods, "Linear
                  contrast-separable shift-invariant imaging systems"),
                  Tikhonov reconstruction (Methods, "Reconstruction
                  algorithm", Eq. tls_solution) and the adjoint.
* ``autotune`` -- mid-band power loss, Adam, finite-difference and analytic
                  parameter gradients (Methods, "Cell-scale optical pooled
                  screen data").
* ``stitch``   -- tiling of a field of view and EDT-weighted blending of the
                  restored tiles (Methods, OPS tiling and stitching).
* ``cnn``      -- the parameter-regression network of the learned initialiser
                  (not in the paper).

Conventions the paper leaves open are fixed once here and listed as
"readings" in the design notes; each function names the reading it uses.

Parity status: every function is pinned by a CPU test against something other
than itself (direct DFT, brute-force convolution, Abbe source summation,
closed-form coherent transfer functions, dense SVD, finite differences),
except the end result of the auto-tune loop, whose parameter error has no
value printed in the paper (parity unpinned; judged against synthetic ground
truth only).
"""

from . import optics, tf, vector, linear, autotune, cnn, stitch  # noqa: F401
