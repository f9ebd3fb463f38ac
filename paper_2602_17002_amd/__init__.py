"""MI355X-native Total Lagrangian internal force, adjoint and tangent kernels."""
