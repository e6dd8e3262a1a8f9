"""FP64 CPU oracle of the SDA camera-fingerprint path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the HIP library
and its Python binding) never imports, links or executes anything here, and
this package imports nothing from the product path.

It is a plain, slow, step-by-step restatement of what the method computes
(arXiv 1909.04573, "Camera Fingerprint Extraction via Spatial Domain Averaged
Frames"), in float64 with NumPy (mpmath for the wavelet filter):

* ``filters``     Daubechies orthonormal low-pass filters (spectral factorisation).
* ``dwt``         periodised separable 2-D analysis / synthesis, multi-level.
* ``wiener``      local-variance Wiener shrinkage (minimum over 3/5/7/9 windows).
* ``sda``         spatial-domain averaged frames (Sec. III-B).
* ``pipeline``    denoiser residual W = I - F(I) (Sec. II-A), MLE fingerprint
                  (Sec. III-A/B), zero-mean, luma, DFT-domain Wiener, query
                  residuals.
* ``correlate``   circular cross-correlation, PCE and NCC (Sec. II-A, Sec. IV).

Where the paper is silent (the denoiser's filter length, boundary handling,
post-processing and PCE details), each function states the reading it takes.
"""
