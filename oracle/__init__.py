"""FP64 CPU oracle for the wavelet-compressed dipole transport.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it reads the seeded inputs from ``synth`` and recomputes everything
(areas, normals, Morton order, SH transfer, the PCA basis, the transport
rows, their Haar transform and top-n truncation, irradiance and radiance)
in plain NumPy float64, following the paper:

* ``dipole``    -- Eq. (4) dipole diffuse reflectance R_d and its derivatives.
* ``geometry``  -- per-vertex areas dA (Eq. 6), normals, 3-D Morton order.
* ``sh``        -- real SH and the unshadowed clamped-cosine transfer
                   (the E(x_i) integral of Eq. 6 / Eq. 11 with V = 1).
* ``pca``       -- the table M and M = USV (Eq. 5, Sec. 2.2), s_k(sigma).
* ``haar``      -- orthonormal Haar transform (Eq. 8; Haar per Sec. 5).
* ``transport`` -- O-A brute-force gather of Eq. (1)-(4) and O-B, the
                   method's discrete operator (Eq. 7, 8 and Step 1 of the
                   precompute in Sec. 3.2; rendering Steps 1-4 of Sec. 4).
* ``adjoint``   -- FP64 adjoint of O-B and its finite-difference check.
* ``cdf97``     -- the CDF 9/7 output-side transform w_1 and its inverse
                   (Sec. 3.2; 9/7 per Sec. 5), filters from their definition.
* ``fresnel``   -- Fresnel transmittance and the outgoing factor
                   (1/pi) F_t(eta, w_o) of Eq. (3) and (6).
* ``spatial``   -- spatial compression of the truncated rows by an energy
                   threshold and its rendering form (Eq. 9, 10; precompute
                   Step 2 of Sec. 3.2; Steps 2, 4, 5 of Sec. 4).

Functions whose result no independent pin covers say "parity unpinned".
"""
