"""Studies of the paper's Secs. IV-V run on lib_llgdisk: static stiffness and
gyrotropic frequency over disk geometries, thermal statistics of the vortex
core, power spectra of <m_x>, and the response to a driven field.

Host-side analysis of what the library returns (fits, histograms, averages)
lives here, outside the library package; every step of the dynamics and
every observable runs in the library's kernels."""
