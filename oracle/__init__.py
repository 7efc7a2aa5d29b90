"""FP64 CPU oracle of the npFEM time step. Test infrastructure only: imported by the tests,
the smoke check and the benchmark's CPU-baseline leg, never by the GPU library."""
from .npfem_oracle import (ARMIJO_C, MAX_HALVINGS, CellType, step, step_batch, predict, gradient, pd_rhs, energy,
                           solve, volume, volume_gradient, surface_area, area_root,
                           triangle_projections, triangle_rest_frames, bending_stencils,
                           bending_vectors, bending_projection, volume_projection,
                           deformation_gradients, interior_edges, system_matrix,
                           cell_volume_area, pbd_damp, rigid_velocity_fit,
                           one_ring_neighbours, median_filter_forces, median_filter_batch,
                           cap_velocities, stiffness_matrix,
                           skalak_density, line_search_update, vertex_normals,
                           closest_foreign_vertex, pik_contacts, packing_step)
