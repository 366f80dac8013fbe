/*
 * lor.h -- C ABI of the MI355X (gfx950) low-order-refined (LOR) assembly library.
 *
 * What is assembled (Pazner, Kolev, Camier, "End-to-end GPU acceleration of
 * low-order-refined preconditioning for high-order finite element
 * discretizations"):
 *   - Section 2.1 (the LOR mesh): each degree-p hexahedron is split at its tensor
 *     Gauss-Lobatto lattice into p^3 trilinear subelements ("macro element").
 *   - Section 2.2: the LOR H1 matrix is the Q1 (p = 1) finite element matrix on
 *     that mesh, here kappa-diffusion + beta-mass, with the same degrees of
 *     freedom as the high-order space.
 *   - Section 2.3: the lowest-order interpolation-histopolation H(curl) case is
 *     the lowest-order Nedelec element on the LOR mesh, here kappa curl-curl +
 *     beta-mass.
 *   - Section 3, Step S1.2 (steps A1 and A2): macro-element assembly followed by
 *     the processor-local CSR matrix (row pointer I, columns J, values A), the
 *     orientation of vector degrees of freedom carried by their sign.
 *
 * Readings of points the paper leaves open: 2x2x2 Gauss-Legendre quadrature per
 * subelement; kappa constant per subelement, beta a scalar; consistent mass;
 * CSR with columns sorted ascending and unique per row, both triangles stored,
 * every structurally present entry kept even where its value cancels.
 *
 * Conventions shared by every call
 *   - Every array argument is a DEVICE pointer (hipMalloc'd / torch CUDA memory)
 *     owned by the caller, except where a parameter says "host".  The library
 *     keeps no device memory between calls; lor_pattern allocates and frees its
 *     own temporaries.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     lor_pattern synchronises `stream` (it must read counts back); the
 *     lor_assemble_* calls are asynchronous on `stream` and never synchronise.
 *   - Status codes are <= 0 (lor_status).  Arguments are validated on the host
 *     before any device work; on error nothing is launched and lor_last_error()
 *     returns a message (thread-local).  No C++ exception crosses the ABI.
 *   - Indices are int32; a mesh whose entry count or nnz reaches 2^31 is
 *     rejected with LOR_EOVERFLOW.
 *   - Results are deterministic: repeated calls give bitwise-identical values,
 *     and A[i][j] and A[j][i] are bitwise equal.
 */
#ifndef LOR_H
#define LOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LOR_OK = 0,
  LOR_EINVAL = -1,        /* bad argument (null pointer, size, p out of range, ...) */
  LOR_EOVERFLOW = -2,     /* an index or count does not fit int32 */
  LOR_EDEVICE = -3,       /* a HIP runtime call failed (message has the HIP error) */
  LOR_EUNSUPPORTED = -4   /* valid input outside what this build handles */
} lor_status;

typedef enum { LOR_H1 = 0, LOR_ND = 1, LOR_RT = 2, LOR_H1_2D = 3 } lor_space;
typedef enum { LOR_F64 = 0, LOR_F32 = 1 } lor_dtype;
/* Diagonal entry of an eliminated row (lor_eliminate_bc). */
typedef enum { LOR_DIAG_ONE = 0, LOR_DIAG_KEEP = 1, LOR_DIAG_ZERO = 2 } lor_diag_policy;

/* Highest polynomial degree handled (the whole macro element is staged in LDS). */
#define LOR_MAX_P 6
/* Most element colours a schedule may use (see lor_sched). */
#define LOR_MAX_COLORS 64
/* Most nonzeros in one row of the assembled matrix. */
#define LOR_MAX_ROW_NNZ 127

/* FP32 form: subelements whose corner-Jacobian ratio max/min exceeds
 * det_ratio_thresh (or whose smallest corner Jacobian is <= 0) are integrated
 * with FP64 geometry instead of FP32. */
#define LOR_FP64_FALLBACK 0x1u
/* lor_assemble_h1, lor_assemble_h1_2d, lor_assemble_rt and lor_assemble_nd:
 * kernel choice.  By default the owner-computes kernel runs when the schedule
 * has it (sched->owner) and the coloured kernel otherwise; LOR_COLORED forces
 * the coloured kernel, LOR_OWNER the owner-computes one (LOR_EUNSUPPORTED if
 * the schedule has none).  Both give the same matrix up to the order of the
 * floating-point sums. */
#define LOR_COLORED 0x2u
#define LOR_OWNER 0x4u

/*
 * Assembly schedule written by lor_pattern and read by the lor_assemble_* calls.
 * The struct itself lives in host memory; `dev` is a caller-owned device
 * buffer of `dev_bytes` bytes that holds the device part:
 *   - the element order by colour (elements of one colour share no degree of
 *     freedom, so one colour is assembled without write conflicts; colours run
 *     in increasing order on the stream),
 *   - per element, for each of its `nent` local stencil entries, the position
 *     of the entry inside its CSR row and whether this element is the first
 *     (lowest colour) contributor to that entry, stored once per distinct
 *     element class (`nclass` classes; on a structured mesh a few hundred, so
 *     the tables the assembly reads stay cache resident),
 *   - the vertex-to-element incidence lists used by the adjoint,
 *   - the reference-element stencil tables (the shared column pattern of one
 *     macro element, computed once, as in step A1).
 * The host fields are descriptive except color_ptr (used to size launches).
 */
typedef struct lor_sched {
  int32_t space;                 /* lor_space */
  int32_t p;
  int64_t nel;
  int64_t nrows;
  int64_t nnz;
  int32_t nloc;                  /* local dofs per element */
  int32_t nent;                  /* local stencil entries per element */
  int32_t ncolors;
  int32_t max_row_nnz;
  int32_t color_ptr[LOR_MAX_COLORS + 1];  /* colour c = order[color_ptr[c] .. color_ptr[c+1]) */
  int64_t nclass;
  int64_t tab_stride;            /* bytes between two element tables (nent rounded up to 16) */
  size_t dev_bytes;              /* written by phase 1: bytes to allocate for dev */
  void* dev;                     /* set by the caller before phase 2 */
  size_t off_order, off_color, off_class, off_tables;
  size_t off_inc_ptr, off_inc_list;
  size_t off_st_ptr, off_st_col, off_ent_row, off_recipe;
  size_t off_zero;               /* 256 zero bytes (read in place of an old value that is absent) */
  size_t off_order_class;        /* class of order[i] (int32 per element, in colour order) */
  /* Owner-computes schedule (LOR_H1, LOR_H1_2D, LOR_RT, LOR_ND; see lor_assemble_h1).  Present
   * (owner == 1) when the mesh is a box lattice: the elements tile a box of
   * box[0] x box[1] x box[2] elements, each with its local axes along the box
   * axes, and the vertex at point (X, Y, Z) of the global lattice of
   * (LX, LY, LZ) = (box[0] p + 1, box[1] p + 1, box[2] p + 1) points has id
   * X + LX (Y + LY Z) -- structured meshes, also with the elements in any
   * order.  Such meshes also get their pattern, colours (by the parities of
   * the box position) and rank tables in closed form.  owner == 0 otherwise,
   * and then only the colour schedule is used.  Phase 1 already sets owner
   * and box (a box lattice needs fewer schedule bytes); phase 2 fills the
   * arrays.  LOR_H1_2D: the same one dimension down (vertex X + LX Y,
   * box[2] = 1, elem3d holds the element at (ex, ey)), found in phase 2 on
   * top of the general schedule, which the coloured kernel keeps using.
   * LOR_RT: a face lattice (see lor_assemble_rt), LOR_ND: an edge lattice
   * (see lor_assemble_nd), both also found in phase 2. */
  size_t off_elem3d;             /* int32 [box[2]][box[1]][box[0]]: element at box position (ex, ey, ez) */
  size_t off_base;               /* int32 [LZ][LY]: vertex id of lattice point (0, Y, Z) */
  int32_t owner;                 /* 1 if the owner-computes schedule is valid */
  int32_t box[3];                /* elements along x, y, z */
  size_t reserved[3];
} lor_sched;

/*
 * lor_pattern -- sparsity pattern (steps A1/A2: the shared local column pattern,
 * row counts, scan, column fill) and the assembly schedule.
 *
 *   space     LOR_H1: rows are mesh vertices; LOR_ND: rows are mesh edges;
 *             LOR_RT: rows are mesh faces; LOR_H1_2D: rows are the vertices
 *             of a 2D (quadrilateral) mesh.
 *   p         polynomial degree, 1 <= p <= LOR_MAX_P.
 *   nel       number of (macro) elements, >= 0.
 *   nrows     number of global dofs (vertices or edges).
 *   elem_map  [nel][nloc] int32.  LOR_H1: nloc = (p+1)^3 global vertex ids,
 *             local vertex i + (p+1)(j + (p+1)k).  LOR_ND: nloc = 3p(p+1)^2
 *             signed global edge ids: x-edges i + p(j + (p+1)k) first, then
 *             y-edges (offset p(p+1)^2, index i + (p+1)(j + p k)), then z-edges
 *             (offset 2p(p+1)^2, index i + (p+1)(j + (p+1)k)); a local edge
 *             points along its +axis; entry v >= 0 is edge v with that
 *             orientation, v < 0 is edge -1-v with the opposite one.
 *             LOR_H1_2D: nloc = (p+1)^2 global vertex ids, local vertex
 *             i + (p+1)j.
 *             LOR_RT: nloc = 3p^2(p+1) signed global face ids, in the layout
 *             and sign convention given at lor_discrete_curl (normals along
 *             +axis locally).
 *   row_ptr   [nrows+1] int32, written in phase 1.
 *   nnz       HOST int64, written in phase 1.
 *   col_idx   NULL selects phase 1.  Otherwise [nnz] int32, written in phase 2
 *             (sorted ascending, unique per row).
 *   sched     HOST struct.  Phase 1 writes sched->dev_bytes; the caller then
 *             sets sched->dev to a device buffer of that size and calls again
 *             with col_idx != NULL (phase 2), which fills the schedule.
 * Phase 1 and phase 2 each synchronise `stream`.  Errors: LOR_EINVAL (bad
 * arguments, a map entry out of [0, nrows), an element whose lattice is not
 * conforming with its neighbours), LOR_EOVERFLOW (nnz or nel*nloc >= 2^31),
 * LOR_EUNSUPPORTED (a row with more than LOR_MAX_ROW_NNZ nonzeros, or more than
 * LOR_MAX_COLORS colours).
 */
int lor_pattern(int space, int p, int64_t nel, int64_t nrows, const int32_t* elem_map,
                int32_t* row_ptr, int64_t* nnz, int32_t* col_idx, lor_sched* sched,
                void* stream);

/*
 * lor_assemble_h1 -- values of the LOR H1 matrix (Section 2.2; Step S1.2 A1+A2):
 *   A = sum over subelements s of  kappa_s K^s + beta M^s,
 *   K^s_uv = sum_q w_q det J (J^-T g_u).(J^-T g_v),  M^s_uv = sum_q w_q det J phi_u phi_v,
 * 2x2x2 Gauss points q on each trilinear subelement.
 *
 *   p, nel, ndofs  as for lor_pattern (space LOR_H1).
 *   batch          number of independent coefficient fields (>= 1).
 *   elem_dofs      [nel][(p+1)^3] int32, the map given to lor_pattern.
 *   coords         [ndofs][3] float64 vertex coordinates (always FP64).
 *   kappa          [batch][nel][p^3] in `dtype`; subelement i + p(j + p k).
 *   beta           mass coefficient (scalar).
 *   row_ptr, sched the pattern and schedule from lor_pattern(LOR_H1, ...).
 *   values         [batch][nnz] in `dtype`, overwritten (every entry written).
 *   dtype          LOR_F64: all arithmetic in FP64.  LOR_F32: edge vectors
 *                  formed in FP64 then rounded; Jacobians, quadrature and
 *                  subelement matrices in FP32 (FP64 on flagged subelements if
 *                  flags has LOR_FP64_FALLBACK); sums within an element in FP64;
 *                  stored as FP32.
 *   flags          LOR_FP64_FALLBACK (FP32 only), and at most one of
 *                  LOR_COLORED / LOR_OWNER (kernel choice, see above).  The
 *                  owner-computes kernel sums every row once, whole, in FP64
 *                  (also in the FP32 form) and stores it once; the coloured
 *                  kernel adds element by element in colour order.
 *   det_ratio_thresh  threshold of the fallback (e.g. 10).
 *   diag           NULL or device int32[2]: [0] += number of subelements that
 *                  took the FP64 fallback, [1] += number of subelements with a
 *                  non-positive Jacobian at a quadrature point (inverted; their
 *                  values are still written).  The caller zeroes it.
 */
int lor_assemble_h1(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                    const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                    const lor_sched* sched, void* values, int dtype, unsigned flags,
                    double det_ratio_thresh, int32_t* diag, void* stream);

/*
 * lor_assemble_nd -- values of the LOR H(curl) matrix (Section 2.3; Step S1.2
 * with orientation signs, A2): lowest-order Nedelec on each subelement,
 *   K_ab = sum_q w det J (J c_a / det J).(J c_b / det J),
 *   M_ab = sum_q w det J (J^-T n_a).(J^-T n_b),
 * times sigma_a sigma_b from the signed edge map; A = kappa_s K + beta M.
 *   elem_dofs   [nel][(p+1)^3] vertex map (geometry).
 *   elem_edges  [nel][3p(p+1)^2] signed edge map (the one given to lor_pattern).
 *   nedges      number of rows.  Other arguments as for lor_assemble_h1.
 * Kernel choice (LOR_COLORED, LOR_OWNER) as for lor_assemble_h1: the
 * owner-computes kernel runs by default when the edge map is an edge lattice
 * (sched->owner: with (MX, MY, MZ) = (box[0] p, box[1] p, box[2] p) cells, the
 * x-edge from lattice point (X, Y, Z) has id X + MX (Y + (MY+1) Z), the
 * y-edges and z-edges follow at OY = MX (MY+1)(MZ+1) and
 * OZ = OY + (MX+1) MY (MZ+1) in the same way, any orientation signs, elements
 * in any order, any vertex numbering); every row is then summed once in FP64
 * and stored once.  The coloured kernel takes p <= 5 (LOR_EUNSUPPORTED
 * above: a macro element's 78 entries per subelement no longer fit in LDS at
 * p = 6); the owner-computes kernel takes every p up to LOR_MAX_P.
 */
int lor_assemble_nd(int p, int64_t nel, int64_t ndofs_h1, int64_t nedges, int batch,
                    const int32_t* elem_dofs, const int32_t* elem_edges, const double* coords,
                    const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                    void* values, int dtype, unsigned flags, double det_ratio_thresh,
                    int32_t* diag, void* stream);

/*
 * lor_assemble_rt -- values of the LOR H(div) matrix (Section 2.3: the
 * lowest-order interpolation-histopolation case is the lowest-order
 * Raviart-Thomas element on the LOR mesh; Step S1.2 with orientation signs,
 * A2): on each subelement, with the contravariant Piola map N = J n / det J,
 *   K_ab = sum_q w det J (div n_a / det J)(div n_b / det J),
 *   M_ab = sum_q w det J (J n_a / det J).(J n_b / det J),
 * times sigma_a sigma_b from the signed face map; A = kappa_s K + beta M.
 *   elem_dofs   [nel][(p+1)^3] vertex map (geometry).
 *   elem_faces  [nel][3p^2(p+1)] signed face map (the one given to lor_pattern
 *               with LOR_RT; layout as at lor_discrete_curl).
 *   nfaces      number of rows.  Other arguments as for lor_assemble_h1.
 * Kernel choice (LOR_COLORED, LOR_OWNER) as for lor_assemble_h1: the
 * owner-computes kernel runs by default when the face map is a face lattice
 * (sched->owner: with (MX, MY, MZ) = (box[0] p, box[1] p, box[2] p) cells, the
 * x-face at lattice x = X of cell row (Y, Z) has id X + (MX+1)(Y + MY Z), the
 * y-faces and z-faces follow at OY = (MX+1) MY MZ and OZ = OY + MX (MY+1) MZ
 * in the same way, any orientation signs, elements in any order, any vertex
 * numbering); every row is then summed once in FP64 and stored once.
 */
int lor_assemble_rt(int p, int64_t nel, int64_t ndofs_h1, int64_t nfaces, int batch,
                    const int32_t* elem_dofs, const int32_t* elem_faces, const double* coords,
                    const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                    void* values, int dtype, unsigned flags, double det_ratio_thresh,
                    int32_t* diag, void* stream);

/*
 * lor_assemble_h1_2d -- values of the 2D LOR H1 matrix (the 2D variant of
 * Step S1.2; Section 4.1 measures it at 9 nonzeros per row): each degree-p
 * quadrilateral macro element is cut at its Gauss-Lobatto lattice into p^2
 * bilinear subelements, and A = sum_s kappa_s K^s + beta M^s with
 *   K_uv = sum_q w det J (J^-T g_u).(J^-T g_v),  M_uv = sum_q w det J phi_u phi_v,
 * 2x2 Gauss points q (w = 1/4) on each subelement.
 *   elem_dofs  [nel][(p+1)^2] vertex ids, local vertex i + (p+1)j.
 *   coords     [ndofs][2] float64.
 *   kappa      [batch][nel][p^2] in dtype, subelement i + p j.
 *   sched      from lor_pattern(LOR_H1_2D, p, elem_dofs).
 * Other arguments, the FP32 form and its fallback (corner-Jacobian ratio of
 * the 4 corners) as for lor_assemble_h1.  Kernel choice (LOR_COLORED,
 * LOR_OWNER) as for lor_assemble_h1: the owner-computes kernel runs by default
 * when the mesh is a 2D box lattice (sched->owner, box[2] = 1; every row is
 * then summed once in FP64 and stored once, in the FP32 form too).
 */
int lor_assemble_h1_2d(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                       const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                       const lor_sched* sched, void* values, int dtype, unsigned flags,
                       double det_ratio_thresh, int32_t* diag, void* stream);

/*
 * lor_refine_map -- the LOR mesh made explicit: every subelement of every
 * macro element becomes an element of its own with 8 vertex ids (the setup the
 * paper's unstructured comparator needs; Section 4, assembly results).
 *   elem_dofs  [nel][(p+1)^3] vertex map.
 *   sub_map    [nel * p^3][8] int32, written: element e p^3 + s (s = i + p(j +
 *              p k)), corner v = a + 2b + 4c -> vertex (i+a, j+b, k+c) of e.
 * Asynchronous on `stream`.  Errors: LOR_EINVAL, LOR_EOVERFLOW.
 */
int lor_refine_map(int p, int64_t nel, const int32_t* elem_dofs, int32_t* sub_map, void* stream);

/*
 * lor_assemble_h1_unstructured -- the generic comparator of Section 4's
 * assembly results: the same H1 LOR matrix (FP64) assembled without the
 * macro-element structure.  One group of 8 lanes per trilinear element, one
 * lane per element dof: the element's 8x8 matrix, then each lane adds its row
 * into the global CSR matrix (position by binary search in the row, FP64
 * atomic add).  The summation order varies between runs (rounding-level
 * differences; not bitwise reproducible, unlike lor_assemble_h1).
 *   nsub, sub_map   [nsub][8] element vertex ids (e.g. from lor_refine_map).
 *   kappa           [nsub] FP64 per element; beta scalar.
 *   row_ptr, col_idx, nnz   the CSR pattern (e.g. lor_pattern of the macro mesh).
 *   values          [nnz] FP64, zeroed then accumulated.
 *   diag            NULL or device int32[2]: [0] += element entries whose
 *                   column is not in the row, or elements with a vertex id
 *                   outside [0, ndofs) (skipped); [1] += elements with
 *                   det J <= 0 at a quadrature point.  The caller zeroes it.
 * Asynchronous on `stream`.  Errors: LOR_EINVAL, LOR_EOVERFLOW.
 */
int lor_assemble_h1_unstructured(int64_t nsub, int64_t ndofs, int64_t nnz, const int32_t* sub_map,
                                 const double* coords, const double* kappa, double beta,
                                 const int32_t* row_ptr, const int32_t* col_idx, double* values,
                                 int32_t* diag, void* stream);

/*
 * lor_assemble_backward -- adjoint of lor_assemble_h1 with respect to kappa and
 * the vertex coordinates, for the loss L = sum_b <grad_values[b], values[b]>:
 *   grad_kappa[b][e][s] = dL/dkappa[b][e][s]                   (overwritten)
 *   grad_coords[v][c]   = sum_b dL/dcoords[v][c]  (FP64, overwritten; coords are
 *                         shared by the batch, so their gradient is summed)
 *   grad_values  [batch][nnz] in dtype;  grad_kappa [batch][nel][p^3] in dtype.
 *   workspace    device buffer of lor_backward_workspace(p, nel, batch, dtype)
 *                bytes (holds the per-element coordinate gradient before the
 *                vertex gather; fully overwritten, needs no clearing).
 * Subelement geometry is recomputed, not stored.  Arithmetic in dtype; the
 * vertex gather sums in FP64 in a fixed order (deterministic).
 */
int lor_assemble_backward(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                          const double* coords, const void* kappa, double beta,
                          const int32_t* row_ptr, const lor_sched* sched, const void* grad_values,
                          void* grad_kappa, double* grad_coords, void* workspace, int dtype,
                          void* stream);

/*
 * lor_assemble_backward_noalloc -- lor_assemble_backward without a workspace
 * argument and without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The per-element coordinate-gradient E-vector lives in a
 * workspace built into the library: one array of
 * lor_backward_noalloc_max_workspace() bytes (32 MiB) per GPU, held from the
 * first call on that GPU until the process ends.  Its contents carry over
 * between calls (every call overwrites the part it reads, so nothing needs
 * clearing); calls that overlap on one GPU (different streams, or host
 * threads) share it and race -- serialise them.
 *   Arguments and results as for lor_assemble_backward.
 *   Errors: as lor_assemble_backward, plus LOR_EUNSUPPORTED when
 *   lor_backward_workspace(p, nel, batch, dtype) exceeds the built-in size
 *   (nel * (p+1)^3 at most 1,398,101), LOR_EDEVICE if the workspace address
 *   cannot be obtained.  No hipMalloc, hipFree or allocating library call.
 */
int lor_assemble_backward_noalloc(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                                  const double* coords, const void* kappa, double beta,
                                  const int32_t* row_ptr, const lor_sched* sched, const void* grad_values,
                                  void* grad_kappa, double* grad_coords, int dtype, void* stream);

/* Bytes of the workspace built into lor_assemble_backward_noalloc (per GPU). */
size_t lor_backward_noalloc_max_workspace(void);

/*
 * lor_eliminate_bc -- elimination of essential boundary conditions from an
 * assembled matrix (Section 3, Step S1.2, step A4), on one device: every entry
 * in the row or the column of an essential dof becomes 0, except the diagonal
 * entry of an essential dof, which becomes 1 (LOR_DIAG_ONE, the usual choice),
 * keeps its value (LOR_DIAG_KEEP) or becomes 0 (LOR_DIAG_ZERO).  In place.
 *
 *   nrows, nnz  matrix size; row_ptr [nrows+1], col_idx [nnz] int32: a CSR
 *               pattern with columns sorted ascending within each row and
 *               structurally symmetric (every (i, j) has a (j, i)), as
 *               lor_pattern writes it.  Column i is found through row i.
 *   values      [batch][nnz] in `dtype` (LOR_F64 or LOR_F32), modified in place.
 *   ess_dofs    [ness] int32 essential dofs, any order, repeats allowed.
 *   marker      [nrows] uint8, written: 1 for an essential dof, else 0 (the
 *               marker array of the paper, e.g. for a right-hand side).
 *   diag        NULL or device int32[2]: [0] += essential entries outside
 *               [0, nrows) (ignored); [1] += column entries (c, i) not found
 *               because the pattern is not structurally symmetric or a column
 *               index is out of range.  The caller zeroes it.
 * Asynchronous on `stream`; writes are deterministic (each entry has one
 * writer).  Errors: LOR_EINVAL (bad sizes, NULL pointers, unknown policy),
 * LOR_EOVERFLOW (nrows, nnz or ness >= 2^31).
 */
int lor_eliminate_bc(int64_t nrows, int64_t nnz, int batch, const int32_t* row_ptr,
                     const int32_t* col_idx, void* values, int dtype, int64_t ness,
                     const int32_t* ess_dofs, uint8_t* marker, int diag_policy, int32_t* diag,
                     void* stream);

/*
 * lor_discrete_gradient -- the discrete gradient matrix G (LOR vertices ->
 * LOR edges) that the auxiliary-space Maxwell solver needs (Section 3, Step
 * S1.2, auxiliary computations, and its algorithm for G in CSR form): row i
 * (edge i) has the two entries I[i] = 2i, J = (first, second) vertex of the
 * edge's local edge in the element that supplies it, A = (-sigma, +sigma) with
 * sigma its orientation sign.  The supplying element is the edge's first
 * incidence (lowest element, then lowest local edge) from the schedule, so
 * the two entries of a row are in that local edge's order, not sorted.
 *
 *   p, nel      as for lor_assemble_nd; ndofs_h1 vertices, nedges edges.
 *   elem_dofs   [nel][(p+1)^3] vertex map; elem_edges the signed edge map.
 *   sched       the schedule lor_pattern(LOR_ND, p, elem_edges) wrote.
 *   row_ptr     [nedges+1] int32, col_idx [2*nedges] int32, values
 *               [2*nedges] in dtype (LOR_F64 / LOR_F32): written.
 *   diag        NULL or device int32[2]: [0] += edges in no element (their row
 *               is two zeros at column 0); [1] += rows with a vertex outside
 *               [0, ndofs_h1).  The caller zeroes it.
 * Asynchronous on `stream`.  Errors: LOR_EINVAL, LOR_EOVERFLOW (2*nedges >= 2^31).
 */
int lor_discrete_gradient(int p, int64_t nel, int64_t ndofs_h1, int64_t nedges, const int32_t* elem_dofs,
                          const int32_t* elem_edges, const lor_sched* sched, int32_t* row_ptr,
                          int32_t* col_idx, void* values, int dtype, int32_t* diag, void* stream);

/*
 * lor_discrete_curl -- the discrete curl matrix C (LOR edges -> LOR faces)
 * that the auxiliary-space divergence solver needs (Section 3, Step S1.2,
 * auxiliary computations): row f (face f) has 4 entries, one per boundary
 * edge of the face, value sigma_f * sigma_e * s with s = +1, +1, -1, -1 the
 * edge's sign in the face's circulation (right-hand rule about the face's
 * +axis normal: x-face boundary +y, +z, -y, -z; y-face +z, +x, -z, -x; z-face
 * +x, +y, -x, -y) on the reference macro element, and sigma_f, sigma_e the
 * signs of the face and edge maps.  Each face is taken from its first
 * incidence (lowest element, then lowest local face); entries stay in that
 * circulation order.
 *
 *   elem_edges  [nel][3p(p+1)^2] signed edge map (as for lor_assemble_nd).
 *   elem_faces  [nel][3p^2(p+1)] signed face map: x-faces (normal +x) first,
 *               local index i + (p+1)(j + p k) with i <= p; then y-faces at
 *               offset p^2(p+1), index i + p(j + (p+1)k) with j <= p; then
 *               z-faces at offset 2p^2(p+1), index i + p(j + p k) with k <= p;
 *               entry f >= 0 is face f with the local orientation, f < 0 is
 *               face -1-f with the opposite one.
 *   workspace   [nfaces] int32 device buffer (first incidence of every face).
 *   row_ptr     [nfaces+1] int32, col_idx [4*nfaces] int32, values [4*nfaces]
 *               in dtype: written.
 *   diag        NULL or device int32[2]: [0] += faces in no element (row of
 *               four zeros at column 0); [1] += face ids >= nfaces in the face
 *               map (ignored) or edge ids >= nedges written.  Caller zeroes it.
 * Asynchronous on `stream`.  Errors: LOR_EINVAL, LOR_EOVERFLOW.
 */
int lor_discrete_curl(int p, int64_t nel, int64_t nedges, int64_t nfaces, const int32_t* elem_edges,
                      const int32_t* elem_faces, int32_t* workspace, int32_t* row_ptr, int32_t* col_idx,
                      void* values, int dtype, int32_t* diag, void* stream);

/*
 * lor_interp_nodes -- LOR vertex coordinates as an E-vector (Section 3,
 * auxiliary computations; the coordinate-vector kernels of Section 4): the
 * degree-q high-order mesh, given by its nodes at the tensor Gauss-Lobatto
 * points of degree q, evaluated at the tensor Gauss-Lobatto lattice of degree
 * p with the tensor-product Lagrange basis (sum-factorised, FP64).
 *
 *   nodes  [nel][(q+1)^3][ncomp] float64, local node i + (q+1)(j + (q+1)k).
 *   out    [nel][(p+1)^3][ncomp] float64, written.
 *   1 <= p <= LOR_MAX_P, 1 <= q <= 8, 1 <= ncomp <= 3.
 * Asynchronous on `stream`.  Errors: LOR_EINVAL, LOR_EOVERFLOW (nel >= 2^31).
 */
int lor_interp_nodes(int p, int q, int64_t nel, int ncomp, const double* nodes, double* out, void* stream);

/*
 * lor_evec_to_tvec -- E-vector to T-vector (the deduplication of the
 * coordinate E-vector with the element restriction map, one thread per dof,
 * Section 3 auxiliary computations): tvec[g] = evec at the first incidence of
 * dof g (lowest element, then lowest local index).
 *
 *   sched  the schedule lor_pattern(LOR_H1, p, elem_dofs) wrote (its incidence
 *          lists give the first incidences).
 *   evec   [nel][(p+1)^3][ncomp] float64; tvec [ndofs][ncomp] float64, written.
 *   diag   NULL or device int32[1]: [0] += dofs in no element (left as 0).
 * Asynchronous on `stream`.  Errors: LOR_EINVAL.
 */
int lor_evec_to_tvec(int p, int64_t nel, int64_t ndofs, const lor_sched* sched, int ncomp, const double* evec,
                     double* tvec, int32_t* diag, void* stream);

/*
 * lor_pattern_workspace -- bytes of the schedule's device buffer (sched->dev)
 * for a mesh of these sizes, known before the pattern is built: an upper
 * bound of the value lor_pattern phase 1 writes into sched->dev_bytes, equal
 * to it unless the mesh is an H1 box lattice (see lor_sched.owner), whose
 * schedule stores fewer rank tables.  0 for invalid arguments (the checks of
 * lor_pattern).  Host only; no device work.
 */
size_t lor_pattern_workspace(int space, int p, int64_t nel, int64_t nrows);

/*
 * lor_backward_workspace -- bytes of the `workspace` argument of
 * lor_assemble_backward for these sizes (the per-element coordinate-gradient
 * E-vector, FP64 [nel][(p+1)^3][3], shared by the batch and by both dtypes).
 * 0 for invalid arguments (p outside [1, LOR_MAX_P], nel < 0, batch < 1,
 * unknown dtype).  Host only.
 */
size_t lor_backward_workspace(int p, int64_t nel, int batch, int dtype);

/* sizeof(lor_sched) as compiled into the library (for bindings to check their layout). */
size_t lor_sched_bytes(void);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* lor_last_error(void);

/* ABI version of this library (incremented on incompatible changes). */
int lor_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LOR_H */
