// Single translation unit for all device code of the PMCHWT library (the
// quadrature tables in constant memory are shared by the assembly, barycentric
// and far-field kernels).
#include "assembly.inl"
#include "bc.inl"
#include "linalg.inl"
#include "mfma.inl"
#include "mfma64.inl"
#include "refine.inl"
#include "massinv.inl"
#include "nearfield.inl"
#include "classify.inl"
