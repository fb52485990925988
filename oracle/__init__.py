"""Plain FP64 CPU oracle of the tiDAS path (arXiv 2507.15464).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the package's
``smoke()`` check and the CPU-baseline leg of the benchmark may import it.
The product path (the HIP library and its Python binding) never imports,
links or calls anything here, and nothing here imports the product path.

Every function is a direct, slow, readable transcription of a definition:

* ``geometry``  element centres, plane-wave transmit delay, receive distance,
                the receive delay law (Sec. 2.1, eqn:delay) and Hann apodization.
* ``pulse``     the transmitted Gaussian-modulated pulse.
* ``simulate``  Born-approximation RF synthesis (Sec. 2, eqn:SRX).
* ``das``       Delay-and-Sum (Sec. 2, eqn:appF), vectorised and brute force.
* ``kernels``   per-depth-row kernels: the exact DAS PSF (Sec. 2.2, eq:PSF)
                and the paper's fixed-delay + least-squares theta kernel
                (Sec. 2.3, eqn:tDAS / eqn:theta; Sec. 3.1-3.2 FWHM window).
* ``tidas``     the per-row convolutional line model (Sec. 2.4,
                eqn:line_conv), its adjoint, its gradient in the kernels and
                its explicit banded matrix.
* ``deconv``    Tikhonov-regularised gradient deconvolution through it.
* ``mlp``       the kernel-surrogate MLP in FP64 and with BF16 rounding
                emulated at the GPU's rounding points.
* ``metrics``   relative errors and the paper's local / global error.
* ``point_study`` the paper's single-point study (Sec. 3.1-3.3): focused
                transmit with a Kossoff aperture, the Theta matrix and the
                local / global error maps of every (delay curve, scatterer)
                pair, and the DAS / tiDAS peak and FWHM along the line.

All arithmetic is float64 (numpy).  Nothing is blocked, fused or reordered
beyond what the definitions state.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, a brute-force loop, a library routine or an invariant; none is
unpinned.
"""
