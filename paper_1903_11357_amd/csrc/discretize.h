// Host-side discretisation of the SIPG problem and of the Schwarz coarse
// transfer (internal to libasdg). Plain C++17, no HIP dependency.
#pragma once

#include <sys/mman.h>

#include <cstdint>
#include <cstdlib>
#include <memory>
#include <new>
#include <functional>
#include <string>
#include <utility>
#include <vector>

namespace asdg {

// Allocator whose resize leaves new elements uninitialised (each user
// writes every element, in parallel, instead of a serial zero fill first).
// Arrays of 4 MiB and more are placed on 2 MiB boundaries with transparent
// huge pages requested: their first touch then faults once per 2 MiB
// instead of once per 4 KiB page (about half the cost of first writing a
// few hundred MB; the request is only advice and is ignored where huge
// pages are off).
template <class T>
struct DefaultInit : std::allocator<T> {
  static constexpr size_t kHuge = size_t(4) << 20, kAlign = size_t(2) << 20;
  template <class U>
  struct rebind {
    using other = DefaultInit<U>;
  };
  DefaultInit() = default;
  template <class U>
  DefaultInit(const DefaultInit<U>&) noexcept {}
  T* allocate(size_t n) {
    const size_t bytes = n * sizeof(T);
    if (bytes < kHuge) return std::allocator<T>::allocate(n);
    void* p = std::aligned_alloc(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
    if (!p) throw std::bad_alloc();
    (void)madvise(p, bytes, MADV_HUGEPAGE);
    return static_cast<T*>(p);
  }
  void deallocate(T* p, size_t n) noexcept {
    if (n * sizeof(T) < kHuge)
      std::allocator<T>::deallocate(p, n);
    else
      std::free(p);
  }
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};

struct Box {
  double x0, x1, y0, y1;
};

struct Box3 {
  double x0, x1, y0, y1, z0, z1;
};

// Polygon mesh view (caller's arrays).
struct MeshView {
  int32_t n_vertices;
  const double* xy;
  int32_t n_cells;
  const int32_t* ptr;
  const int32_t* verts;
};

// Gauss-Legendre rule with m points on [0, 1] (weights sum to one).
void gauss_legendre01(int m, std::vector<double>& x, std::vector<double>& w);

// Highest polynomial degree of the 2D assembly and its basis size.
constexpr int kMaxDegree2D = 9;
constexpr int kMaxBasis2D = (kMaxDegree2D + 1) * (kMaxDegree2D + 2) / 2;

// Scaled Legendre basis of total degree p on box B: basis_prepare computes
// the box's factors (centre, scalings, normalisations) once, basis_eval the
// n_p values and gradients (either may be null) at a point.
int n_basis(int p);
struct BasisBox {
  int p;
  double dx, dy, cx, cy, sx, sy;
  double s[kMaxBasis2D];
};
void basis_prepare(int p, const Box& B, BasisBox& bb);
void basis_eval(const BasisBox& bb, double x, double y, double* val, double* gx, double* gy);

struct CellGeom {
  std::vector<double> area, cx, cy, diam;
  std::vector<Box> box;
};

struct Face {
  int32_t plus, minus;  // minus < 0: boundary face
  int32_t v0, v1;       // endpoints in the plus cell's CCW order
};

// SIPG system in the internal (subdomain-major) cell order.
struct Assembled {
  int p = 0, np = 0;
  double c_sigma = 0.0;
  int32_t n_cells = 0, n_sub = 0;
  std::vector<int32_t> perm;     // internal cell -> caller cell
  std::vector<int32_t> iperm;    // caller cell -> internal cell
  std::vector<int32_t> sub_ptr;  // [n_sub + 1] internal cell offsets
  std::vector<int32_t> row_ptr;  // BSR, internal order
  std::vector<int32_t> col_idx;
  std::vector<double, DefaultInit<double>> blocks;  // per block np*np, element (a,b) at a*np + b (row-major)
  std::vector<double> rhs;       // internal order
  CellGeom geom;                 // caller order (2D)
  std::vector<Face> faces;       // caller cell ids (2D)
  int dim = 2;
  std::vector<Box3> box3;        // caller order (3D)
  std::vector<double> diam3;     // caller order (3D)
};

// Returns empty string on success, otherwise an error message.
std::string assemble_sipg(const MeshView& mesh, int p, double c_sigma, const double* rho,
                          const int32_t* subdomain,
                          void (*f)(int64_t, const double*, double*, void*), void* f_user,
                          Assembled& out);

// Coarse transfer P_0 (internal fine order), CSR by fine cell with np x nq
// blocks (row-major, element (a,c) at a*nq + c), and the Galerkin A_0.
struct Coarse {
  int q = 0, nq = 0;
  int32_t n_coarse = 0;
  std::vector<int32_t> ptr;     // [n_cells + 1]
  std::vector<int32_t> col;     // coarse cell of each block
  std::vector<double> val;      // blocks
  std::vector<int32_t> tptr;    // [n_coarse + 1] transposed lists
  std::vector<int32_t> tcell;   // fine (internal) cell of each entry
  std::vector<int32_t> tblk;    // block index into col/val
  std::vector<double, DefaultInit<double>> a0;  // dense n0 x n0 row-major
};

std::string build_coarse(const MeshView& fine, const Assembled& A, int q,
                         const int32_t* coarse_of_cell, const MeshView* coarse_mesh, Coarse& out);

// ---- 3D: tetrahedral meshes (discretize3.cpp)
// Tetrahedral mesh view (caller's arrays): tets [n_cells][4] vertex ids.
struct TetView {
  int32_t n_vertices;
  const double* xyz;
  int32_t n_cells;
  const int32_t* tets;
};

// Scaled Legendre basis of total degree p on a box, ordered by degree d,
// then k = 0..d, then j = 0..d-k, i = d-j-k (exponents of x, y, z).
// basis_prepare3 computes the box's factors once, basis_eval3 the values and
// gradients (either may be null) at a point.
int n_basis3(int p);
struct BasisBox3 {
  int p;
  double d[3], c[3], sc[3];
  double s[20];
};
void basis_prepare3(int p, const Box3& B, BasisBox3& bb);
void basis_eval3(const BasisBox3& bb, double x, double y, double z, double* val, double* gx, double* gy,
                 double* gz);

// 3D SIPG system; fills out.box3 / out.diam3 (caller order) and sets out.dim = 3.
std::string assemble_sipg_tet(const TetView& mesh, int p, double c_sigma, const double* rho,
                              const int32_t* subdomain,
                              void (*f)(int64_t, const double*, double*, void*), void* f_user, Assembled& out);

// Nested coarse transfer for agglomerates of tetrahedra (coarse_of_cell).
std::string build_coarse_tet(const TetView& fine, const Assembled& A, int q, const int32_t* coarse_of_cell,
                             Coarse& out);

// ---- shared by the 2D and 3D builders (internal)
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn);

// Caps the threads parallel_for starts from the calling thread while the
// object lives (0 = the default: hardware threads, at most 16).
class HostThreadCap {
 public:
  explicit HostThreadCap(int n);
  ~HostThreadCap();

 private:
  int prev_;
};
bool spd_solve(int n, std::vector<double> M, double* B, int k);
std::string finish_assembly(Assembled& A, const int32_t* subdomain, const std::vector<std::pair<int32_t, int32_t>>& pm,
                            const double* vol, const double* rhs_c, const double* fblk);
void finish_coarse(const Assembled& A, const std::vector<std::vector<int32_t>>& bcol,
                   const std::vector<std::vector<double>>& bval, Coarse& C);

}  // namespace asdg
