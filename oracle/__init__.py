"""CPU oracle for the regularised Biot-Savart FMM (test infrastructure only).

Plain, slow, double-precision reference implementations written from the
paper (Yokota & Barba, "FMM-based vortex method for simulation of isotropic
turbulence on GPUs, compared with a spectral method"):

* ``direct``    -- the defining O(N^2) sums of eqs. 5-8 (C + OpenMP, and a
                   NumPy twin for tiny cases), free space or cubic image
                   blocks of the periodic cube;
* ``tree``      -- Morton keys, stable sort, leaf ranges, neighbour and
                   interaction lists of the uniform octree, by brute force;
* ``harmonics`` -- spherical harmonics and the multipole/local operators in
                   the nomenclature of Cheng et al. that the paper uses
                   (eqs. 10-11) and their translation theorems;
* ``fmm``       -- the FMM evaluation of u and grad u (eqs. 12-15) built from
                   those pieces, including the periodic lattice sum;
* ``spectral``  -- the infinite-lattice velocity of lattice-placed Gaussian
                   blobs by FFT (used to check the periodic sums).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library.
"""
