"""Seeded synthetic inputs (meshes, cell mixes, placements, forces) shared by the oracle
tests and the GPU library's callers. Holds no solver arithmetic."""
from .meshes import (rbc_mesh, platelet_mesh, tetrahedron, octahedron, icosahedron, bipyramid,
                     uv_sphere_topology, mesh_summary, RBC_DIAMETER, PLT_DIAMETER)
from .workloads import (DT, RBC, PLT, DIAMETER, Material, RBC_MATERIAL, PLT_MATERIAL,
                        cell_type_inputs, make_batch, force_stream, strong_cells, Batch,
                        Workload, WORKLOADS, random_rotations, NOMINAL_VOLUME, PACKING,
                        packing_batch)
