"""Plain FP64 CPU oracle for the per-candidate MoM evaluation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library never calls it and shares no code with it.

What it computes, for a pixel map and a frequency (paper Section II):

* ``geometry``  -- the pixel mesh (two triangles per pixel, alternating
  diagonals), the feeds and vias, and the RWG basis functions with their
  classification into always-present, inner-pixel, inter-pixel and pixel-port
  functions (Section II-C, Fig. 2(a)).
* ``singular``  -- closed-form potential integrals over a flat triangle used to
  extract the 1/R singularity of the Green's function.
* ``efie``      -- the impedance matrix of the EFIE (Eq. 1) expanded in RWG
  functions (Eq. 2), mixed-potential form, homogeneous medium.
* ``network``   -- the selection of Eqs. 3-5, the dense solve of Eq. 2 and the
  S-parameters of Eqs. 6-7.
* ``fom``       -- the figure of merit of Eqs. 8-9.
* ``search``    -- the single-flip sweep and the accept rule of Algorithm 1.

Parity status per function is stated in each module header.
"""
